// BF16 form of the interpolant contraction Y = [Phi | P] W (Eq. rbfcoeff):
// kernel rows and weights rounded to bfloat16, products accumulated in FP32 on
// v_mfma_f32_16x16x32_bf16 (lane l holds A[l%16][8(l/16) + e] and
// B[8(l/16) + e][l%16], e < 8; accumulator element i = D[4(l/16) + i][l%16],
// measured on gfx950).  An 8-bit significand cannot carry the interpolant's
// cancellation (sum_r |B_r W_rc| exceeds the result by 1e4 or more), so this
// form exists to report its error, not to meet the ln L tolerance.
//
// Memory layout (8-row groups g, G8 = rows / 8): rows AB[g][q][8], weights
// WB[g][c][8], 16 bytes per (group, proposal or column).  A workgroup of 4
// waves (2 x 2) computes 64 proposals x 64 columns, each wave 2 x 2 tiles of
// 16 x 16; 32-row steps of both operands staged through LDS, double-buffered.
#include "basis_rows.h"
#include "rbfl_internal.h"

namespace rbfl {

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

constexpr int kBfThreads = 256;

__device__ __forceinline__ v4i pack_bf16(const double *v) {
  bf8 b;
#pragma unroll
  for (int e = 0; e < 8; ++e) b[e] = (__bf16)(float)v[e];
  return __builtin_bit_cast(v4i, b);
}

// Rows 8g .. 8g + 7 of proposal q; thread t = g * nb + q.
__global__ void __launch_bounds__(256) k_rows_bf16(const EvalConsts *__restrict__ cp,
                                                   const double *__restrict__ params, int64_t ld, int64_t b0,
                                                   int64_t nb, const double *__restrict__ nodes,
                                                   v4i *__restrict__ AB) {
  const EvalConsts &c = *cp;
  const int G8 = c.rows / 8;
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= (int64_t)G8 * nb) return;
  const int g = (int)(t / nb);
  const int64_t q = t - (int64_t)g * nb;
  double x[4];
#pragma unroll
  for (int d = 0; d < 4; ++d) x[d] = params[d * ld + b0 + q] / c.semi[d];
  const int N = c.N, NM = c.N + c.M;
  double v[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int r = 8 * g + k;
    v[k] = basis_row_fp64(r, N, NM, x, nodes + 4 * (int64_t)r, c.eps2, c.poly_idx);
  }
  AB[t] = pack_bf16(v);
}

// Weights in the same grouped layout; thread t = g * Kp + col.
__global__ void __launch_bounds__(256) k_weights_bf16(const double *__restrict__ W, int rows, int Kp,
                                                      v4i *__restrict__ WB) {
  const int G8 = rows / 8;
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= (int64_t)G8 * Kp) return;
  const int g = (int)(t / Kp), col = (int)(t - (int64_t)g * Kp);
  double v[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) v[k] = W[(int64_t)(8 * g + k) * Kp + col];
  WB[t] = pack_bf16(v);
}

// Workgroups are dealt to the 8 XCDs in turn; this gives each XCD a
// contiguous range of logical tiles (a bijection for any grid size), so the
// column tiles of one proposal tile run on one XCD and share its L2.
__device__ __forceinline__ int64_t xcd_logical_block(int64_t b, int64_t nblk) {
  const int64_t x = b & 7, slot = b >> 3, base = nblk >> 3, extra = nblk & 7;
  return x * base + (x < extra ? x : extra) + slot;
}

__global__ void __launch_bounds__(kBfThreads, 2)
    k_bf16_contract(const v4i *__restrict__ AB, int64_t nb, int rows, const v4i *__restrict__ WB, int Kp,
                    double *__restrict__ Y) {
  __shared__ v4i As[2][4][64];
  __shared__ v4i Bs[2][4][64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wq = wave & 1, wc = wave >> 1;
  const int n_ct = Kp / 64;
  const int64_t tile = xcd_logical_block(blockIdx.x, gridDim.x);
  const int c0 = (int)(tile % n_ct) * 64;
  const int64_t q0 = (tile / n_ct) * 64;
  // staging: entry tid = (group within the step, proposal or column)
  const int sg = tid >> 6, sm = tid & 63;
  const bool in_q = q0 + sm < nb;
  v4i ra, rb;
  auto fetch = [&](int g0) {
    ra = in_q ? AB[(int64_t)(g0 + sg) * nb + q0 + sm] : v4i{0, 0, 0, 0};
    rb = WB[(int64_t)(g0 + sg) * Kp + c0 + sm];
  };
  auto stash = [&](int buf) {
    // keeps the compiler from hoisting these LDS writes (and the wait for
    // their global loads) above the current step's MFMAs
    asm volatile("" ::: "memory");
    As[buf][sg][sm] = ra;
    Bs[buf][sg][sm] = rb;
  };
  f4 acc[2][2];
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int u = 0; u < 2; ++u) acc[t][u] = f4{0.0f, 0.0f, 0.0f, 0.0f};
  const int n_steps = rows / 32;
  const int kg = lane >> 4, ll = lane & 15;
  fetch(0);
  stash(0);
  __syncthreads();
  for (int st = 0; st < n_steps; ++st) {
    const int cur = st & 1;
    if (st + 1 < n_steps) fetch(4 * (st + 1));
    bf8 a[2], b[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) a[t] = __builtin_bit_cast(bf8, As[cur][kg][wq * 32 + 16 * t + ll]);
#pragma unroll
    for (int u = 0; u < 2; ++u) b[u] = __builtin_bit_cast(bf8, Bs[cur][kg][wc * 32 + 16 * u + ll]);
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int u = 0; u < 2; ++u) acc[t][u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[t], b[u], acc[t][u], 0, 0, 0);
    if (st + 1 < n_steps) stash(cur ^ 1);
    __syncthreads();
  }
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t q = q0 + wq * 32 + 16 * t + 4 * kg + i;
      if (q >= nb) continue;
#pragma unroll
      for (int u = 0; u < 2; ++u) Y[q * Kp + c0 + wc * 32 + 16 * u + ll] = (double)acc[t][u][i];
    }
}

}  // namespace

void launch_bf16_prepare(const double *W, int rows, int Kp, uint16_t *WB, hipStream_t s) {
  const int64_t n = (int64_t)(rows / 8) * Kp;
  hipLaunchKernelGGL(k_weights_bf16, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, W, rows, Kp,
                     reinterpret_cast<v4i *>(WB));
  RBFL_HIP(hipGetLastError());
}

void launch_contract_bf16(const EvalConsts *c, const EvalConsts &hc, const double *params, int64_t ld, int64_t b0,
                          int64_t nb, const double *nodes, uint16_t *AB, const uint16_t *WB, double *Y,
                          hipStream_t s, hipEvent_t mid) {
  static_assert(kRowChunk % 32 == 0 && kColTile % 64 == 0, "K and the rows are padded to whole tiles");
  const int64_t G8 = hc.rows / 8;
  hipLaunchKernelGGL(k_rows_bf16, dim3((unsigned)((G8 * nb + 255) / 256)), dim3(256), 0, s, c, params, ld, b0, nb,
                     nodes, reinterpret_cast<v4i *>(AB));
  RBFL_HIP(hipGetLastError());
  if (mid) RBFL_HIP(hipEventRecord(mid, s));
  const int64_t nblk = (nb + 63) / 64 * (hc.Kp / 64);
  hipLaunchKernelGGL(k_bf16_contract, dim3((unsigned)nblk), dim3(kBfThreads), 0, s,
                     reinterpret_cast<const v4i *>(AB), nb, hc.rows, reinterpret_cast<const v4i *>(WB), hc.Kp, Y);
  RBFL_HIP(hipGetLastError());
}

}  // namespace rbfl
