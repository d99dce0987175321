// FP64 form of the interpolant contraction Y = [Phi | P] W (Eq. rbfcoeff) as
// two kernels: the basis rows of a chunk of proposals are written to HBM by a
// VALU-only kernel, then a DGEMM-shaped FP64 MFMA kernel contracts them with
// the weights.
//
// Why not fused: on gfx950 an FP64 MFMA and any VALU instruction of the same
// SIMD do not execute concurrently (the co-execution counter stays at zero),
// so the ~45 VALU instructions of each fused exp(-eps^2 d^2) row value (plus
// its recomputation for every column tile) are added to the MFMA time.  Apart
// from the rows the GEMM's inner loop issues only LDS reads and MFMAs; the
// rows cost one HBM round trip of 8 (N + M) bytes per proposal.
//
// Layouts: rows Bt[r][q] (row r of proposal q, leading dimension ldb, a
// multiple of 8 >= nb, zero beyond nb); weights W[r][c] (Kp columns).
// GEMM tiles: 4 waves (2 x 2), each RT x CT tiles of 16 x 16 on
// v_mfma_f64_16x16x4f64 (lane l holds A[l%16][l/16], B[l/16][l%16];
// accumulator element i is D[l/16 + 4i][l%16], measured on gfx950); row
// chunks of KC rows of both operands staged through LDS, double-buffered.
#include "basis_rows.h"
#include "epilogue_setup.h"
#include "rbfl_internal.h"

namespace rbfl {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef double d2 __attribute__((ext_vector_type(2)));

constexpr int kGemmThreads = 256;

// Basis rows 16*blockIdx.y .. +15 of proposals q = blockIdx.x*256 + tid (zero
// for nb <= q < ldb).
__global__ void __launch_bounds__(256) k_rows_fp64(const EvalConsts *__restrict__ cp,
                                                   const double *__restrict__ params, int64_t ld, int64_t b0,
                                                   int64_t nb, int64_t ldb, const double *__restrict__ nodes,
                                                   double *__restrict__ Bt) {
  const EvalConsts &c = *cp;
  const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (q >= ldb) return;
  const int r0 = 16 * blockIdx.y;
  if (q >= nb) {
#pragma unroll
    for (int k = 0; k < 16; ++k) Bt[(int64_t)(r0 + k) * ldb + q] = 0.0;
    return;
  }
  double x[4];
#pragma unroll
  for (int d = 0; d < 4; ++d) x[d] = params[d * ld + b0 + q] / c.semi[d];
  const int N = c.N, NM = c.N + c.M;
#pragma unroll 4
  for (int k = 0; k < 16; ++k) {
    const int r = r0 + k;
    Bt[(int64_t)r * ldb + q] = basis_row_fp64(r, N, NM, x, nodes + 4 * (int64_t)r, c.eps2, c.poly_idx);
  }
}

// Workgroups are dealt to the 8 XCDs in turn; this gives each XCD a
// contiguous range of logical tiles (a bijection for any grid size), so the
// column tiles of one proposal tile run on one XCD and share its L2.
__device__ __forceinline__ int64_t xcd_logical_block(int64_t b, int64_t nblk) {
  const int64_t x = b & 7, slot = b >> 3, base = nblk >> 3, extra = nblk & 7;
  return x * base + (x < extra ? x : extra) + slot;
}

// One output tile of Y[q][c] = sum_r Bt[r][q] W[r][c]: proposals tq*QT ..,
// columns tc*CW ..; called by every thread of the workgroup.
template <int RT, int CT, int KC, int WQ = 2, int WC = 2>
__device__ __forceinline__ void gemm_tile(const double *__restrict__ Bt, int64_t nb, int64_t ldb, int rows,
                                          const double *__restrict__ W, int Kp, double *__restrict__ Y, int64_t tq,
                                          int tc) {
  constexpr int QT = WQ * RT * 16, CW = WC * CT * 16, NT = 64 * WQ * WC;
  constexpr int A2 = KC * QT / 2, W2 = KC * CW / 2;                 // double2 entries per chunk
  constexpr int LA = A2 / NT, LW = W2 / NT;
  static_assert(KC % 4 == 0 && A2 % NT == 0 && W2 % NT == 0, "whole k-steps, even staging");
  __shared__ double As[2][KC][QT];
  __shared__ double Ws[2][KC][CW];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wq = wave % WQ, wc = wave / WQ;
  const int c0 = tc * CW;
  const int64_t q0 = tq * QT;

  // per-thread source pointers of the staged entries, advanced by KC rows per chunk
  const double *pa[LA];
  const double *pw[LW];
  bool va[LA];
#pragma unroll
  for (int u = 0; u < LA; ++u) {
    const int e = tid + u * NT;
    const int k = e / (QT / 2), q2 = e % (QT / 2);
    pa[u] = Bt + (int64_t)k * ldb + q0 + 2 * q2;
    va[u] = q0 + 2 * q2 < ldb;
  }
#pragma unroll
  for (int u = 0; u < LW; ++u) {
    const int e = tid + u * NT;
    pw[u] = W + (int64_t)(e / (CW / 2)) * Kp + c0 + 2 * (e % (CW / 2));
  }
  const int64_t stepA = (int64_t)KC * ldb, stepW = (int64_t)KC * Kp;
  d2 ra[LA], rw[LW];
  auto fetch = [&]() {
#pragma unroll
    for (int u = 0; u < LA; ++u) {
      ra[u] = va[u] ? *reinterpret_cast<const d2 *>(pa[u]) : d2{0.0, 0.0};
      pa[u] += stepA;
    }
#pragma unroll
    for (int u = 0; u < LW; ++u) {
      rw[u] = *reinterpret_cast<const d2 *>(pw[u]);
      pw[u] += stepW;
    }
  };
  auto stash = [&](int buf) {
    // keeps the compiler from hoisting these LDS writes (and the wait for
    // their global loads) above the current chunk's MFMAs
    asm volatile("" ::: "memory");
#pragma unroll
    for (int u = 0; u < LA; ++u) {
      const int e = tid + u * NT;
      *reinterpret_cast<d2 *>(&As[buf][e / (QT / 2)][2 * (e % (QT / 2))]) = ra[u];
    }
#pragma unroll
    for (int u = 0; u < LW; ++u) {
      const int e = tid + u * NT;
      *reinterpret_cast<d2 *>(&Ws[buf][e / (CW / 2)][2 * (e % (CW / 2))]) = rw[u];
    }
  };

  d4 acc[RT][CT];
#pragma unroll
  for (int t = 0; t < RT; ++t)
#pragma unroll
    for (int u = 0; u < CT; ++u) acc[t][u] = d4{0.0, 0.0, 0.0, 0.0};

  const int kk = lane >> 4, ll = lane & 15;
  const int n_chunks = rows / KC;
  fetch();
  stash(0);
  __syncthreads();
  for (int ch = 0; ch < n_chunks; ++ch) {
    const int cur = ch & 1;
    if (ch + 1 < n_chunks) fetch();
#pragma unroll
    for (int s = 0; s < KC / 4; ++s) {
      const int k = 4 * s + kk;
      double a[RT], b[CT];
#pragma unroll
      for (int t = 0; t < RT; ++t) a[t] = As[cur][k][wq * RT * 16 + 16 * t + ll];
#pragma unroll
      for (int u = 0; u < CT; ++u) b[u] = Ws[cur][k][wc * CT * 16 + 16 * u + ll];
#pragma unroll
      for (int t = 0; t < RT; ++t)
#pragma unroll
        for (int u = 0; u < CT; ++u) acc[t][u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[t], b[u], acc[t][u], 0, 0, 0);
    }
    if (ch + 1 < n_chunks) stash(cur ^ 1);
    __syncthreads();
  }
#pragma unroll
  for (int t = 0; t < RT; ++t)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t q = q0 + wq * RT * 16 + 16 * t + kk + 4 * i;
      if (q >= nb) continue;
#pragma unroll
      for (int u = 0; u < CT; ++u) Y[q * Kp + c0 + wc * CT * 16 + 16 * u + ll] = acc[t][u][i];
    }
}

// One-dimensional grid over (proposal tile, column tile), column tile fastest;
// WQ x WC waves per workgroup.
template <int RT, int CT, int KC, int WQ, int WC>
__global__ void __launch_bounds__(64 * WQ * WC, 512 / (64 * WQ * WC))
    k_gemm_fp64(const double *__restrict__ Bt, int64_t nb, int64_t ldb, int rows, const double *__restrict__ W,
                int Kp, double *__restrict__ Y) {
  const int n_ct = Kp / (WC * CT * 16);
  const int64_t tile = xcd_logical_block(blockIdx.x, gridDim.x);
  gemm_tile<RT, CT, KC, WQ, WC>(Bt, nb, ldb, rows, W, Kp, Y, tile / n_ct, (int)(tile % n_ct));
}

// The accumulators of one output tile of Y[q][c] = sum_r Bt[r][q] W[r][c]
// (the K loop of gemm_tile, kept as a copy so that gemm_tile's code is not
// changed by this kernel):
// proposals tq*QT .., columns tc*CW ..; called by every thread of the
// workgroup; acc[t][u][i] of lane l is Y at proposal
// tq*QT + (wave % WQ)*RT*16 + 16t + l/16 + 4i and column
// tc*CW + (wave / WQ)*CT*16 + 16u + l%16.
template <int RT, int CT, int KC, int WQ = 2, int WC = 2>
__device__ __forceinline__ void gemm_accumulate(const double *__restrict__ Bt, int64_t ldb, int rows,
                                                const double *__restrict__ W, int Kp, int64_t tq, int tc,
                                                d4 (&acc)[RT][CT]) {
  constexpr int QT = WQ * RT * 16, CW = WC * CT * 16, NT = 64 * WQ * WC;
  constexpr int A2 = KC * QT / 2, W2 = KC * CW / 2;                 // double2 entries per chunk
  constexpr int LA = A2 / NT, LW = W2 / NT;
  static_assert(KC % 4 == 0 && A2 % NT == 0 && W2 % NT == 0, "whole k-steps, even staging");
  __shared__ double As[2][KC][QT];
  __shared__ double Ws[2][KC][CW];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wq = wave % WQ, wc = wave / WQ;
  const int c0 = tc * CW;
  const int64_t q0 = tq * QT;

  // per-thread source pointers of the staged entries, advanced by KC rows per chunk
  const double *pa[LA];
  const double *pw[LW];
  bool va[LA];
#pragma unroll
  for (int u = 0; u < LA; ++u) {
    const int e = tid + u * NT;
    const int k = e / (QT / 2), q2 = e % (QT / 2);
    pa[u] = Bt + (int64_t)k * ldb + q0 + 2 * q2;
    va[u] = q0 + 2 * q2 < ldb;
  }
#pragma unroll
  for (int u = 0; u < LW; ++u) {
    const int e = tid + u * NT;
    pw[u] = W + (int64_t)(e / (CW / 2)) * Kp + c0 + 2 * (e % (CW / 2));
  }
  const int64_t stepA = (int64_t)KC * ldb, stepW = (int64_t)KC * Kp;
  d2 ra[LA], rw[LW];
  auto fetch = [&]() {
#pragma unroll
    for (int u = 0; u < LA; ++u) {
      ra[u] = va[u] ? *reinterpret_cast<const d2 *>(pa[u]) : d2{0.0, 0.0};
      pa[u] += stepA;
    }
#pragma unroll
    for (int u = 0; u < LW; ++u) {
      rw[u] = *reinterpret_cast<const d2 *>(pw[u]);
      pw[u] += stepW;
    }
  };
  auto stash = [&](int buf) {
    // keeps the compiler from hoisting these LDS writes (and the wait for
    // their global loads) above the current chunk's MFMAs
    asm volatile("" ::: "memory");
#pragma unroll
    for (int u = 0; u < LA; ++u) {
      const int e = tid + u * NT;
      *reinterpret_cast<d2 *>(&As[buf][e / (QT / 2)][2 * (e % (QT / 2))]) = ra[u];
    }
#pragma unroll
    for (int u = 0; u < LW; ++u) {
      const int e = tid + u * NT;
      *reinterpret_cast<d2 *>(&Ws[buf][e / (CW / 2)][2 * (e % (CW / 2))]) = rw[u];
    }
  };

#pragma unroll
  for (int t = 0; t < RT; ++t)
#pragma unroll
    for (int u = 0; u < CT; ++u) acc[t][u] = d4{0.0, 0.0, 0.0, 0.0};

  const int kk = lane >> 4, ll = lane & 15;
  const int n_chunks = rows / KC;
  fetch();
  stash(0);
  __syncthreads();
  for (int ch = 0; ch < n_chunks; ++ch) {
    const int cur = ch & 1;
    if (ch + 1 < n_chunks) fetch();
#pragma unroll
    for (int s = 0; s < KC / 4; ++s) {
      const int k = 4 * s + kk;
      double a[RT], b[CT];
#pragma unroll
      for (int t = 0; t < RT; ++t) a[t] = As[cur][k][wq * RT * 16 + 16 * t + ll];
#pragma unroll
      for (int u = 0; u < CT; ++u) b[u] = Ws[cur][k][wc * CT * 16 + 16 * u + ll];
#pragma unroll
      for (int t = 0; t < RT; ++t)
#pragma unroll
        for (int u = 0; u < CT; ++u) acc[t][u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[t], b[u], acc[t][u], 0, 0, 0);
    }
    if (ch + 1 < n_chunks) stash(cur ^ 1);
    __syncthreads();
  }
}

// The FP64 contraction that finishes ln L itself.  ln L is linear in the
// interpolated outputs, ln L = sum_c w_c Y[c], with the weights w_c of
// lnl_weight (the terms of Eq. logl_complete, corrected reading, as the
// epilogue kernel sums them).  After the same accumulation as k_gemm_fp64's
// 128 x 128 tile of 8 waves, each lane weights its 32 outputs, the 16 lanes
// of a row group and the two column waves add theirs (a fixed tree), and the
// tile writes one partial sum per proposal to part[column tile][proposal];
// Y is never written.  Proposals outside the domain contribute nothing here.
constexpr int kLnlRT = 2, kLnlCT = 4, kLnlKC = 8, kLnlWQ = 4, kLnlWC = 2;

__global__ void __launch_bounds__(64 * kLnlWQ * kLnlWC, 1)
    k_gemm_lnl_fp64(const double *__restrict__ Bt, int64_t nb, int64_t ldb, int rows, const double *__restrict__ W,
                    int Kp, const EvalConsts *__restrict__ cp, const EpiSetup *__restrict__ setups,
                    const double2 *__restrict__ basis4, const int4 *__restrict__ coldesc, double *__restrict__ part,
                    int64_t ldp) {
  constexpr int RT = kLnlRT, CT = kLnlCT, WQ = kLnlWQ, WC = kLnlWC;
  constexpr int QT = WQ * RT * 16, CW = WC * CT * 16;
  __shared__ double red[WC][QT];
  const int n_ct = Kp / CW;
  const int64_t tile = xcd_logical_block(blockIdx.x, gridDim.x);
  const int64_t tq = tile / n_ct;
  const int tc = (int)(tile % n_ct);
  d4 acc[RT][CT];
  gemm_accumulate<RT, CT, kLnlKC, WQ, WC>(Bt, ldb, rows, W, Kp, tq, tc, acc);
  const EvalConsts &c = *cp;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wq = wave % WQ, wc = wave / WQ, kk = lane >> 4, ll = lane & 15;
  const int n_modes = c.n_modes, T = c.T, q = c.q, K = c.K;
  const int64_t q0 = tq * QT;
  int4 dsc[CT];
#pragma unroll
  for (int u = 0; u < CT; ++u) {
    const int j = tc * CW + wc * CT * 16 + 16 * u + ll;
    dsc[u] = j < K ? coldesc[j] : make_int4(-1, 0, 0, 0);
  }
#pragma unroll
  for (int t = 0; t < RT; ++t)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int row = wq * RT * 16 + 16 * t + kk + 4 * i;
      const int64_t b = q0 + row;
      double sum = 0.0;
      if (b < nb && setups[b].status == 0) {
        const EpiSetup &o = setups[b];
#pragma unroll
        for (int u = 0; u < CT; ++u) {
          const int4 d = dsc[u];
          if (d.x < 0) continue;
          sum = fma(lnl_weight(d, o, n_modes, T, q, basis4), acc[t][u][i], sum);
        }
      }
#pragma unroll
      for (int m = 8; m >= 1; m >>= 1) sum += __shfl_xor(sum, m, 64);
      if (ll == 0) red[wc][row] = sum;
    }
  __syncthreads();
  for (int r = threadIdx.x; r < QT; r += 64 * WQ * WC) {
    const int64_t b = q0 + r;
    if (b >= nb) continue;
    double v = red[0][r];
#pragma unroll
    for (int w = 1; w < WC; ++w) v += red[w][r];
    part[(int64_t)tc * ldp + b] = v;
  }
}

// Multi-event batches: basis rows of every event in one launch.  blockIdx.y
// runs over the 16-row groups of all events (event e owns groups rg0 ..);
// blockIdx.x * 256 + tid is the proposal within the event.
__global__ void __launch_bounds__(256) k_ragged_rows_fp64(const EventDesc *__restrict__ ev, int n_ev,
                                                          const double *__restrict__ params, int64_t ld) {
  const int64_t gy = blockIdx.y;
  int lo = 0, hi = n_ev - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (ev[mid].rg0 <= gy) lo = mid;
    else hi = mid - 1;
  }
  const EventDesc &d = ev[lo];
  const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (q >= d.ldb) return;
  const int r0 = 16 * (int)(gy - d.rg0);
  if (q >= d.n) {
#pragma unroll
    for (int k = 0; k < 16; ++k) d.Bt[(int64_t)(r0 + k) * d.ldb + q] = 0.0;
    return;
  }
  const EvalConsts &c = *d.consts;
  double x[4];
#pragma unroll
  for (int dd = 0; dd < 4; ++dd) x[dd] = params[dd * ld + d.q0 + q] / c.semi[dd];
  const int N = c.N, NM = c.N + c.M;
#pragma unroll 4
  for (int k = 0; k < 16; ++k) {
    const int r = r0 + k;
    d.Bt[(int64_t)r * d.ldb + q] = basis_row_fp64(r, N, NM, x, d.nodes + 4 * (int64_t)r, c.eps2, c.poly_idx);
  }
}

// Persistent GEMM over the work list of every event: items are (event,
// proposal tile, column tile), column tile fastest within an event, events in
// the caller's cost order; each workgroup takes the next item from an atomic
// counter until the list is exhausted (every workgroup reaches that exit).
template <int RT, int CT, int KC, int WQ = 2, int WC = 2>
__global__ void __launch_bounds__(64 * WQ * WC, 512 / (64 * WQ * WC))
    k_ragged_gemm_fp64(const EventDesc *__restrict__ ev, int n_ev, int64_t total_items,
                       unsigned long long *__restrict__ counter) {
  __shared__ long long item_s;
  for (;;) {
    if (threadIdx.x == 0) item_s = (long long)atomicAdd(counter, 1ull);
    __syncthreads();
    const int64_t item = item_s;
    __syncthreads();
    if (item >= total_items) break;
    const EventDesc &d = ev[work_event(ev, n_ev, item)];
    const int64_t local = item - d.item0;
    gemm_tile<RT, CT, KC, WQ, WC>(d.Bt, d.n, d.ldb, d.rows, d.W, d.Kp, d.Y, local / d.tiles_c,
                                  (int)(local % d.tiles_c));
  }
}

__global__ void k_zero_item_counter(unsigned long long *counter) {
  if (threadIdx.x == 0) *counter = 0ull;
}

// Rows the GEMMs contract: N + M rounded up to their chunk of KC rows.  The
// padded rows up to hc.rows hold zeros in W (and in the basis rows), so the
// chunks past this bound would only add zeros: the result is the same.
int gemm_rows(const EvalConsts &hc, int kc) { return (hc.N + hc.M + kc - 1) / kc * kc; }

// Basis rows that k_rows_fp64 writes: N + M rounded up to its 16-row groups
// (at least gemm_rows for chunks of 8 or 16 rows).
int basis_rows_written(const EvalConsts &hc) { return (hc.N + hc.M + 15) / 16 * 16; }

template <int RT, int CT, int KC, int WQ = 2, int WC = 2>
void launch_gemm(const double *Bt, int64_t nb, int64_t ldb, const EvalConsts &hc, const double *W, double *Y,
                 hipStream_t s) {
  constexpr int QT = WQ * RT * 16, CW = WC * CT * 16;
  static_assert(kColTile % CW == 0 && kRowChunk % KC == 0 && 16 % KC == 0, "K and the rows are padded to whole tiles");
  const int64_t nblk = (nb + QT - 1) / QT * (hc.Kp / CW);
  hipLaunchKernelGGL((k_gemm_fp64<RT, CT, KC, WQ, WC>), dim3((unsigned)nblk), dim3(64 * WQ * WC), 0, s, Bt, nb, ldb,
                     gemm_rows(hc, KC), W, hc.Kp, Y);
  RBFL_HIP(hipGetLastError());
}

}  // namespace

int64_t rows_ld(int64_t n) { return (n + 7) & ~int64_t(7); }

int gemm_lnl_col_tile() { return kLnlWC * kLnlCT * 16; }

void launch_gemm_lnl_fp64(const double *Bt, int64_t nb, const EvalConsts &hc, const double *W, const EvalConsts *c,
                          const void *setups, const double2 *basis4, const int4 *coldesc, double *part, int64_t ldp,
                          hipStream_t s) {
  constexpr int QT = kLnlWQ * kLnlRT * 16, CW = kLnlWC * kLnlCT * 16;
  static_assert(kColTile % CW == 0 && kRowChunk % kLnlKC == 0, "K and the rows are padded to whole tiles");
  if (nb <= 0) return;
  const int64_t ldb = rows_ld(nb);
  const int64_t nblk = (nb + QT - 1) / QT * (hc.Kp / CW);
  hipLaunchKernelGGL(k_gemm_lnl_fp64, dim3((unsigned)nblk), dim3(64 * kLnlWQ * kLnlWC), 0, s, Bt, nb, ldb,
                     gemm_rows(hc, kLnlKC), W,
                     hc.Kp, c, static_cast<const EpiSetup *>(setups), basis4, coldesc, part, ldp);
  RBFL_HIP(hipGetLastError());
}

int gemm_fp64_variants() { return 7; }

const char *gemm_fp64_variant_name(int v) {
  static const char *names[] = {"rows + gemm 64x128 kc8",  "rows + gemm 128x64 kc8", "rows + gemm 64x128 kc16",
                                "rows + gemm 128x64 kc16", "rows + gemm 64x64 kc8",
                                "rows + gemm 256x128 kc8 (8 waves)", "rows + gemm 128x128 kc8 (8 waves)"};
  return names[v];
}

// Operand reuse of a variant's workgroup tile, QT CW / (QT + CW): the
// algorithmic bytes over the bytes the workgroups read, up to a constant.
double gemm_fp64_reuse(int v) {
  static const double qt[] = {64, 128, 64, 128, 64, 256, 128}, cw[] = {128, 64, 128, 64, 64, 128, 128};
  return qt[v] * cw[v] / (qt[v] + cw[v]);
}

void launch_rows_fp64(const EvalConsts *c, const EvalConsts &hc, const double *params, int64_t ld, int64_t b0,
                      int64_t nb, const double *nodes, double *Bt, hipStream_t s) {
  const int64_t ldb = rows_ld(nb);
  dim3 grid((unsigned)((ldb + 255) / 256), (unsigned)(basis_rows_written(hc) / 16));
  hipLaunchKernelGGL(k_rows_fp64, grid, dim3(256), 0, s, c, params, ld, b0, nb, ldb, nodes, Bt);
  RBFL_HIP(hipGetLastError());
}

void launch_ragged_rows_fp64(const EventDesc *ev, int n_ev, int64_t total_groups, int64_t max_ldb,
                             const double *params, int64_t ld, hipStream_t s) {
  dim3 grid((unsigned)((max_ldb + 255) / 256), (unsigned)total_groups);
  hipLaunchKernelGGL(k_ragged_rows_fp64, grid, dim3(256), 0, s, ev, n_ev, params, ld);
  RBFL_HIP(hipGetLastError());
}

// Multi-event GEMM tiles: variant 0 is 64 x 128 with 8-row chunks (4 waves),
// variant 1 64 x 128 with 16-row chunks (4 waves), variant 2 128 x 128 with
// 8-row chunks (8 waves, the single-event kernel's preferred tile).
void launch_ragged_gemm_fp64(int variant, const EventDesc *ev, int n_ev, int64_t total_items,
                             unsigned long long *counter, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_item_counter, dim3(1), dim3(64), 0, s, counter);
  RBFL_HIP(hipGetLastError());
  if (variant == 2)
    hipLaunchKernelGGL((k_ragged_gemm_fp64<2, 4, 8, 4, 2>), dim3(grid), dim3(512), 0, s, ev, n_ev, total_items,
                       counter);
  else if (variant == 1)
    hipLaunchKernelGGL((k_ragged_gemm_fp64<2, 4, 16>), dim3(grid), dim3(kGemmThreads), 0, s, ev, n_ev, total_items,
                       counter);
  else
    hipLaunchKernelGGL((k_ragged_gemm_fp64<2, 4, 8>), dim3(grid), dim3(kGemmThreads), 0, s, ev, n_ev, total_items,
                       counter);
  RBFL_HIP(hipGetLastError());
}

void launch_gemm_fp64(const double *Bt, int64_t nb, const EvalConsts &hc, const double *W, double *Y, hipStream_t s,
                      int variant) {
  const int64_t ldb = rows_ld(nb);
  switch (variant) {
    case 0: launch_gemm<2, 4, 8>(Bt, nb, ldb, hc, W, Y, s); break;
    case 1: launch_gemm<4, 2, 8>(Bt, nb, ldb, hc, W, Y, s); break;
    case 2: launch_gemm<2, 4, 16>(Bt, nb, ldb, hc, W, Y, s); break;
    case 3: launch_gemm<4, 2, 16>(Bt, nb, ldb, hc, W, Y, s); break;
    case 4: launch_gemm<2, 2, 8>(Bt, nb, ldb, hc, W, Y, s); break;
    case 5: launch_gemm<4, 4, 8, 4, 2>(Bt, nb, ldb, hc, W, Y, s); break;
    case 6: launch_gemm<2, 4, 8, 4, 2>(Bt, nb, ldb, hc, W, Y, s); break;
    default: throw Error(RBFL_E_INVALID_ARG, "unknown FP64 GEMM variant");
  }
}

}  // namespace rbfl
