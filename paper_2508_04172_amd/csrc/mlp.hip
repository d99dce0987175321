// Surrogate network kernels: a multilayer perceptron in -> H -> H -> out with
// SiLU activations, trained by the project's own forward, backward and Adam
// kernels (FP32 arithmetic on the FP32 matrix cores, FP32 master weights).
//
// Parameter layout: W1 [H][in], b1 [H], W2 [H][H], b2 [H], W3 [out][H],
// b3 [out], weights row-major.  Initialisation from caller-provided standard
// normal deviates z: W = z / sqrt(fan_in), b = 0.
#include "rbfl_internal.h"

namespace rbfl {

namespace {

constexpr int kT = 256;

typedef float f4 __attribute__((ext_vector_type(4)));

// C[m][n] = act(sum_k A(m,k) B(k,n) + bias[n]) with A(m,k) = A[m*sam + k*sak]
// and B(k,n) = B[k*sbk + n*sbn] (strides express the transposes).  64x64
// tile per block, 16-deep k chunks through LDS; 4 waves (2 x 2), each 2 x 2
// tiles of 16 x 16 on v_mfma_f32_16x16x4f32 (lane l holds A[l%16][l/16] and
// B[l/16][l%16]; accumulator element i is D[4(l/16) + i][l%16], measured on
// gfx950).  With Z != nullptr the pre-activation is stored too.
template <int ACT>
__global__ void __launch_bounds__(kT) k_gemm_f32(int M, int N, int K, const float *__restrict__ A, int64_t sam,
                                                 int64_t sak, const float *__restrict__ B, int64_t sbk, int64_t sbn,
                                                 const float *__restrict__ bias, float *__restrict__ Z,
                                                 float *__restrict__ C, int64_t ldc) {
  __shared__ float As[16][64 + 4];
  __shared__ float Bs[16][64 + 4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wq = wave & 1, wc = wave >> 1;
  const int kk = lane >> 4, ll = lane & 15;
  // one-dimensional grid, column tile fastest; workgroups are dealt to the 8
  // XCDs in turn, so logical tiles are remapped to give each XCD a contiguous
  // range: the column tiles of one row tile share an XCD's L2 (and its rows
  // of A are fetched from HBM once)
  const int n_nt = (N + 63) / 64;
  const int64_t nblk = gridDim.x, bx = blockIdx.x;
  const int64_t xcd = bx & 7, slot = bx >> 3, base = nblk >> 3, extra = nblk & 7;
  const int64_t tile = xcd * base + (xcd < extra ? xcd : extra) + slot;
  const int m0 = (int)(tile / n_nt) * 64, n0 = (int)(tile % n_nt) * 64;
  f4 acc[2][2];
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int u = 0; u < 2; ++u) acc[t][u] = f4{0.0f, 0.0f, 0.0f, 0.0f};
  // staging: consecutive threads walk the operand's contiguous dimension (k
  // when its k stride is 1, else m or n), so that a wave's loads coalesce
  const bool a_k = sak == 1, b_k = sbk == 1;
  for (int k0 = 0; k0 < K; k0 += 16) {
    for (int e = tid; e < 16 * 64; e += kT) {
      const int ek = a_k ? (e & 15) : (e >> 6), em = a_k ? (e >> 4) : (e & 63);
      const int m = m0 + em, k = k0 + ek;
      As[ek][em] = (m < M && k < K) ? A[(int64_t)m * sam + (int64_t)k * sak] : 0.0f;
    }
    for (int e = tid; e < 16 * 64; e += kT) {
      const int ek = b_k ? (e & 15) : (e >> 6), en = b_k ? (e >> 4) : (e & 63);
      const int n = n0 + en, k = k0 + ek;
      Bs[ek][en] = (n < N && k < K) ? B[(int64_t)k * sbk + (int64_t)n * sbn] : 0.0f;
    }
    __syncthreads();
#pragma unroll
    for (int st = 0; st < 4; ++st) {
      const int k = 4 * st + kk;
      float a[2], b[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) a[t] = As[k][wq * 32 + 16 * t + ll];
#pragma unroll
      for (int u = 0; u < 2; ++u) b[u] = Bs[k][wc * 32 + 16 * u + ll];
#pragma unroll
      for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int u = 0; u < 2; ++u) acc[t][u] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[t], b[u], acc[t][u], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int m = m0 + wq * 32 + 16 * t + 4 * kk + i;
      if (m >= M) continue;
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int n = n0 + wc * 32 + 16 * u + ll;
        if (n >= N) continue;
        float v = acc[t][u][i] + (bias ? bias[n] : 0.0f);
        if (Z) Z[(int64_t)m * ldc + n] = v;
        if (ACT == 1) v = v / (1.0f + __expf(-v));
        C[(int64_t)m * ldc + n] = v;
      }
    }
}

// Forward layers whose operands are both contiguous in k (activations
// A[m][k], weights W[n][k]): 128 x 128 tiles of 8 waves (4 along m x 2 along
// n, each 2 x 4 tiles of 16 x 16), 16-deep k chunks double-buffered through
// LDS with one float4 of each operand per thread and chunk, the same
// XCD-aware tile order.  The accumulation runs over k in the order of
// k_gemm_f32 (chunks of 16, MFMA steps of 4), so the results are the same;
// the caller guarantees K % 16 == 0 and 16-byte aligned rows.
// ACT 0: linear, 1: SiLU, 2: linear with the output standardisation undone
// in FP64, Y[m][n] = mu[n] + sd[n] v into the interpolant's output layout
// (row stride ldc), as the surrogate form's inference needs it; with Bb set
// (residual form) the FP64 polynomial base sum_j Ub[m][j] Bb[j][n] is added
// (Ub: the proposal's nbase monomials, Bb: the base coefficients [nbase][N]).
template <int ACT>
__global__ void __launch_bounds__(512) k_gemm_f32_nt(int M, int N, int K, const float *__restrict__ A, int64_t lda,
                                                     const float *__restrict__ B, int64_t ldb,
                                                     const float *__restrict__ bias, float *__restrict__ Z,
                                                     float *__restrict__ C, int64_t ldc, const float *__restrict__ mu,
                                                     const float *__restrict__ sd, double *__restrict__ Y64,
                                                     const double *__restrict__ Ub, const double *__restrict__ Bb,
                                                     int nbase) {
  __shared__ float As[2][16][128 + 4];
  __shared__ float Bs[2][16][128 + 4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wq = wave & 3, wc = wave >> 2;
  const int kk = lane >> 4, ll = lane & 15;
  const int n_nt = (N + 127) / 128;
  const int64_t nblk = gridDim.x, bx = blockIdx.x;
  const int64_t xcd = bx & 7, slot = bx >> 3, base = nblk >> 3, extra = nblk & 7;
  const int64_t tile = xcd * base + (xcd < extra ? xcd : extra) + slot;
  const int m0 = (int)(tile / n_nt) * 128, n0 = (int)(tile % n_nt) * 128;
  // staging: thread tid carries row tid / 4 of both tiles, k quad (tid % 4) * 4
  const int sr = tid >> 2, sk = (tid & 3) * 4;
  const int am = m0 + sr, bn = n0 + sr;
  const float *pa = A + (int64_t)(am < M ? am : 0) * lda + sk;
  const float *pb = B + (int64_t)(bn < N ? bn : 0) * ldb + sk;
  f4 ra, rb;
  auto fetch = [&](int k0) {
    ra = am < M ? *reinterpret_cast<const f4 *>(pa + k0) : f4{0.0f, 0.0f, 0.0f, 0.0f};
    rb = bn < N ? *reinterpret_cast<const f4 *>(pb + k0) : f4{0.0f, 0.0f, 0.0f, 0.0f};
  };
  auto stash = [&](int buf) {
    asm volatile("" ::: "memory");
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      As[buf][sk + j][sr] = ra[j];
      Bs[buf][sk + j][sr] = rb[j];
    }
  };
  f4 acc[2][4];
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int u = 0; u < 4; ++u) acc[t][u] = f4{0.0f, 0.0f, 0.0f, 0.0f};
  const int n_chunks = K / 16;
  fetch(0);
  stash(0);
  __syncthreads();
  for (int ch = 0; ch < n_chunks; ++ch) {
    const int cur = ch & 1;
    if (ch + 1 < n_chunks) fetch(16 * (ch + 1));
#pragma unroll
    for (int st = 0; st < 4; ++st) {
      const int k = 4 * st + kk;
      float a[2], b[4];
#pragma unroll
      for (int t = 0; t < 2; ++t) a[t] = As[cur][k][wq * 32 + 16 * t + ll];
#pragma unroll
      for (int u = 0; u < 4; ++u) b[u] = Bs[cur][k][wc * 64 + 16 * u + ll];
#pragma unroll
      for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int u = 0; u < 4; ++u) acc[t][u] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[t], b[u], acc[t][u], 0, 0, 0);
    }
    if (ch + 1 < n_chunks) stash(cur ^ 1);
    __syncthreads();
  }
  // residual form: this thread's 2 x 4 rows x 4 columns of the FP64 base
  double bsum[2][4][4] = {};
  if (ACT == 2 && Bb) {
    for (int j = 0; j < nbase; ++j) {
      double uj[2][4], bj[4];
#pragma unroll
      for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int m = m0 + wq * 32 + 16 * t + 4 * kk + i;
          uj[t][i] = m < M ? Ub[(int64_t)m * nbase + j] : 0.0;
        }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int n = n0 + wc * 64 + 16 * u + ll;
        bj[u] = n < N ? Bb[(int64_t)j * N + n] : 0.0;
      }
#pragma unroll
      for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int u = 0; u < 4; ++u) bsum[t][i][u] = fma(uj[t][i], bj[u], bsum[t][i][u]);
    }
  }
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int m = m0 + wq * 32 + 16 * t + 4 * kk + i;
      if (m >= M) continue;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int n = n0 + wc * 64 + 16 * u + ll;
        if (n >= N) continue;
        float v = acc[t][u][i] + (bias ? bias[n] : 0.0f);
        if (ACT == 2) {
          Y64[(int64_t)m * ldc + n] = (double)mu[n] + (double)sd[n] * (double)v + bsum[t][i][u];
          continue;
        }
        if (Z) Z[(int64_t)m * ldc + n] = v;
        if (ACT == 1) v = v / (1.0f + __expf(-v));
        C[(int64_t)m * ldc + n] = v;
      }
    }
}

// Y[b][c] = mu[c] + sd[c] y[b][c] in FP64 (row stride ldy) from FP32 y [B][out],
// plus the FP64 base sum_j Ub[b][j] Bb[j][c] of the residual form when Bb is set.
__global__ void __launch_bounds__(kT) k_unstandardise(const float *__restrict__ y, int64_t B, int out,
                                                      const float *__restrict__ mu, const float *__restrict__ sd,
                                                      double *__restrict__ Y, int64_t ldy,
                                                      const double *__restrict__ Ub, const double *__restrict__ Bb,
                                                      int nbase) {
  const int64_t e = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (e >= B * out) return;
  const int64_t b = e / out;
  const int c = (int)(e - b * out);
  double base = 0.0;
  if (Bb)
    for (int j = 0; j < nbase; ++j) base = fma(Ub[b * nbase + j], Bb[(int64_t)j * out + c], base);
  Y[b * ldy + c] = (double)mu[c] + (double)sd[c] * (double)y[e] + base;
}

// dY = 2 (Y - T) / count; per-block partial sums of (Y - T)^2 (fixed order).
__global__ void __launch_bounds__(kT) k_mse(const float *__restrict__ Y, const float *__restrict__ T, int64_t n,
                                            float scale, float *__restrict__ dY, double *__restrict__ part) {
  __shared__ double red[kT];
  double s = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * kT + threadIdx.x; e < n; e += (int64_t)gridDim.x * kT) {
    const float r = Y[e] - T[e];
    dY[e] = 2.0f * r * scale;
    s += (double)r * (double)r;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = kT / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void k_sum_parts(const double *__restrict__ part, int n, double scale, double *__restrict__ out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += part[i];
    *out = s * scale;
  }
}

// dZ = dH * silu'(Z), silu'(z) = s (1 + z (1 - s)), s = 1 / (1 + e^-z).
__global__ void k_silu_back(const float *__restrict__ dH, const float *__restrict__ Z, int64_t n,
                            float *__restrict__ dZ) {
  const int64_t e = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (e >= n) return;
  const float z = Z[e];
  const float s = 1.0f / (1.0f + __expf(-z));
  dZ[e] = dH[e] * s * (1.0f + z * (1.0f - s));
}

// db[n] = sum_b dZ[b][n].
__global__ void k_colsum(const float *__restrict__ dZ, int B, int N, float *__restrict__ db) {
  const int n = blockIdx.x * kT + threadIdx.x;
  if (n >= N) return;
  float s = 0.0f;
  for (int b = 0; b < B; ++b) s += dZ[(int64_t)b * N + n];
  db[n] = s;
}

__global__ void k_adam(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, int64_t n, float lr, float b1, float b2, float eps, float bc1,
                       float bc2) {
  const int64_t e = (int64_t)blockIdx.x * kT + threadIdx.x;
  if (e >= n) return;
  const float ge = g[e];
  const float me = b1 * m[e] + (1.0f - b1) * ge;
  const float ve = b2 * v[e] + (1.0f - b2) * ge * ge;
  m[e] = me;
  v[e] = ve;
  p[e] -= lr * (me / bc1) / (sqrtf(ve / bc2) + eps);
}

inline unsigned blocks(int64_t n) { return (unsigned)((n + kT - 1) / kT); }

}  // namespace

void Mlp::init(int n_in, int hidden, int n_out, const double *normals) {
  in = n_in;
  hid = hidden;
  out = n_out;
  o_w1 = 0;
  o_b1 = o_w1 + (int64_t)hid * in;
  o_w2 = o_b1 + hid;
  o_b2 = o_w2 + (int64_t)hid * hid;
  o_w3 = o_b2 + hid;
  o_b3 = o_w3 + (int64_t)out * hid;
  np = o_b3 + out;
  std::vector<float> h(np, 0.0f);
  for (int64_t i = 0; i < (int64_t)hid * in; ++i) h[o_w1 + i] = (float)(normals[o_w1 + i] / sqrt((double)in));
  for (int64_t i = 0; i < (int64_t)hid * hid; ++i) h[o_w2 + i] = (float)(normals[o_w2 + i] / sqrt((double)hid));
  for (int64_t i = 0; i < (int64_t)out * hid; ++i) h[o_w3 + i] = (float)(normals[o_w3 + i] / sqrt((double)hid));
  p.alloc(np);
  g.alloc(np);
  m.alloc(np);
  v.alloc(np);
  RBFL_HIP(hipMemcpy(p.p, h.data(), sizeof(float) * np, hipMemcpyHostToDevice));
  RBFL_HIP(hipMemset(g.p, 0, sizeof(float) * np));
  RBFL_HIP(hipMemset(m.p, 0, sizeof(float) * np));
  RBFL_HIP(hipMemset(v.p, 0, sizeof(float) * np));
  loss.alloc(1);
  t = 0;
}

void Mlp::reserve(int64_t B) {
  if (B <= cap) return;
  Z1.alloc((size_t)B * hid);
  H1.alloc((size_t)B * hid);
  Z2.alloc((size_t)B * hid);
  H2.alloc((size_t)B * hid);
  Yb.alloc((size_t)B * out);
  dY.alloc((size_t)B * out);
  dA.alloc((size_t)B * hid);
  dB.alloc((size_t)B * hid);
  part.alloc(1024);
  cap = B;
}

// Whether k_gemm_f32_nt applies: both operands contiguous in k, K a multiple
// of its 16-deep chunks, rows of 16-byte aligned float4s.
static bool nt_ok(int K, const float *A, int64_t sam, int64_t sak, const float *B, int64_t sbk, int64_t sbn) {
  const bool aligned = ((reinterpret_cast<uintptr_t>(A) | reinterpret_cast<uintptr_t>(B)) & 15) == 0;
  return sak == 1 && sbk == 1 && K % 16 == 0 && sam % 4 == 0 && sbn % 4 == 0 && aligned;
}

static void gemm(int act, int M, int N, int K, const float *A, int64_t sam, int64_t sak, const float *B, int64_t sbk,
                 int64_t sbn, const float *bias, float *Z, float *C, int64_t ldc, hipStream_t s) {
  if (nt_ok(K, A, sam, sak, B, sbk, sbn)) {
    dim3 g((unsigned)((int64_t)((N + 127) / 128) * ((M + 127) / 128)));
    if (act)
      hipLaunchKernelGGL(k_gemm_f32_nt<1>, g, dim3(512), 0, s, M, N, K, A, sam, B, sbn, bias, Z, C, ldc, nullptr,
                         nullptr, nullptr, nullptr, nullptr, 0);
    else
      hipLaunchKernelGGL(k_gemm_f32_nt<0>, g, dim3(512), 0, s, M, N, K, A, sam, B, sbn, bias, Z, C, ldc, nullptr,
                         nullptr, nullptr, nullptr, nullptr, 0);
    RBFL_HIP(hipGetLastError());
    return;
  }
  dim3 grid((unsigned)((int64_t)((N + 63) / 64) * ((M + 63) / 64)));
  if (act)
    hipLaunchKernelGGL(k_gemm_f32<1>, grid, dim3(kT), 0, s, M, N, K, A, sam, sak, B, sbk, sbn, bias, Z, C, ldc);
  else
    hipLaunchKernelGGL(k_gemm_f32<0>, grid, dim3(kT), 0, s, M, N, K, A, sam, sak, B, sbk, sbn, bias, Z, C, ldc);
  RBFL_HIP(hipGetLastError());
}

void Mlp::forward(const float *X, int64_t B, float *Y, hipStream_t s) {
  reserve(B);
  const int b = (int)B;
  gemm(1, b, hid, in, X, in, 1, p.p + o_w1, 1, in, p.p + o_b1, Z1.p, H1.p, hid, s);
  gemm(1, b, hid, hid, H1.p, hid, 1, p.p + o_w2, 1, hid, p.p + o_b2, Z2.p, H2.p, hid, s);
  gemm(0, b, out, hid, H2.p, hid, 1, p.p + o_w3, 1, hid, p.p + o_b3, nullptr, Y, out, s);
}

void Mlp::infer(const float *X, int64_t B, const float *mu, const float *sd, double *Y, int64_t ldy, hipStream_t s,
                const double *Ub, const double *Bb, int nbase) {
  reserve(B);
  const int b = (int)B;
  gemm(1, b, hid, in, X, in, 1, p.p + o_w1, 1, in, p.p + o_b1, nullptr, H1.p, hid, s);
  gemm(1, b, hid, hid, H1.p, hid, 1, p.p + o_w2, 1, hid, p.p + o_b2, nullptr, H2.p, hid, s);
  const float *W3 = p.p + o_w3;
  if (nt_ok(hid, H2.p, hid, 1, W3, 1, hid)) {
    dim3 g((unsigned)((int64_t)((out + 127) / 128) * ((b + 127) / 128)));
    hipLaunchKernelGGL(k_gemm_f32_nt<2>, g, dim3(512), 0, s, b, out, hid, H2.p, (int64_t)hid, W3, (int64_t)hid,
                       p.p + o_b3, nullptr, nullptr, ldy, mu, sd, Y, Ub, Bb, nbase);
    RBFL_HIP(hipGetLastError());
    return;
  }
  gemm(0, b, out, hid, H2.p, hid, 1, W3, 1, hid, p.p + o_b3, nullptr, Yb.p, out, s);
  hipLaunchKernelGGL(k_unstandardise, dim3((unsigned)(((int64_t)b * out + kT - 1) / kT)), dim3(kT), 0, s, Yb.p,
                     (int64_t)b, out, mu, sd, Y, ldy, Ub, Bb, nbase);
  RBFL_HIP(hipGetLastError());
}

void Mlp::loss_grad(const float *X, const float *T, int64_t B, hipStream_t s) {
  reserve(B);
  const int b = (int)B;
  forward(X, B, Yb.p, s);
  const int64_t n = B * out;
  const int nblk = (int)std::min<int64_t>(1024, (n + kT - 1) / kT);
  hipLaunchKernelGGL(k_mse, dim3(nblk), dim3(kT), 0, s, Yb.p, T, n, (float)(1.0 / (double)n), dY.p, part.p);
  RBFL_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(64), 0, s, part.p, nblk, 1.0 / (double)n, loss.p);
  RBFL_HIP(hipGetLastError());
  // layer 3: dW3 = dY^T H2, db3 = colsum dY, dH2 = dY W3
  gemm(0, out, hid, b, dY.p, 1, out, H2.p, hid, 1, nullptr, nullptr, g.p + o_w3, hid, s);
  hipLaunchKernelGGL(k_colsum, dim3(blocks(out)), dim3(kT), 0, s, dY.p, b, out, g.p + o_b3);
  RBFL_HIP(hipGetLastError());
  gemm(0, b, hid, out, dY.p, out, 1, p.p + o_w3, hid, 1, nullptr, nullptr, dA.p, hid, s);
  hipLaunchKernelGGL(k_silu_back, dim3(blocks((int64_t)b * hid)), dim3(kT), 0, s, dA.p, Z2.p, (int64_t)b * hid, dB.p);
  RBFL_HIP(hipGetLastError());
  // layer 2: dW2 = dZ2^T H1, db2, dH1 = dZ2 W2
  gemm(0, hid, hid, b, dB.p, 1, hid, H1.p, hid, 1, nullptr, nullptr, g.p + o_w2, hid, s);
  hipLaunchKernelGGL(k_colsum, dim3(blocks(hid)), dim3(kT), 0, s, dB.p, b, hid, g.p + o_b2);
  RBFL_HIP(hipGetLastError());
  gemm(0, b, hid, hid, dB.p, hid, 1, p.p + o_w2, hid, 1, nullptr, nullptr, dA.p, hid, s);
  hipLaunchKernelGGL(k_silu_back, dim3(blocks((int64_t)b * hid)), dim3(kT), 0, s, dA.p, Z1.p, (int64_t)b * hid, dB.p);
  RBFL_HIP(hipGetLastError());
  // layer 1: dW1 = dZ1^T X, db1
  gemm(0, hid, in, b, dB.p, 1, hid, X, in, 1, nullptr, nullptr, g.p + o_w1, in, s);
  hipLaunchKernelGGL(k_colsum, dim3(blocks(hid)), dim3(kT), 0, s, dB.p, b, hid, g.p + o_b1);
  RBFL_HIP(hipGetLastError());
}

void Mlp::adam(double lr, double b1, double b2, double eps, hipStream_t s) {
  ++t;
  const float bc1 = (float)(1.0 - pow(b1, t)), bc2 = (float)(1.0 - pow(b2, t));
  hipLaunchKernelGGL(k_adam, dim3(blocks(np)), dim3(kT), 0, s, p.p, g.p, m.p, v.p, np, (float)lr, (float)b1,
                     (float)b2, (float)eps, bc1, bc2);
  RBFL_HIP(hipGetLastError());
}

}  // namespace rbfl
