// Split form of the interpolant contraction Y = [Phi | P] W (Eq. rbfcoeff)
// on the int8 matrix cores, exact up to the truncation of its operands.
//
// Digits.  A real v with |v| <= 1 is written in signed base-254 digits,
//   v = sum_i a_i u_i + rest,  u_i = 1 / (127 * 254^i),  |a_i| <= 127,
// a_0 = rint(127 v), then repeatedly r <- 254 r - a_i (one FMA, remainder in
// [-1/2, 1/2]) and a_{i+1} = rint(254 r).  After S digits |rest| <= u_{S-1}/2
// = 254^-S (the FMA rounding adds ~2^-54 of a digit unit per step).  The
// digits of a value do not depend on S: the weights are cut once into
// kMaxSlices digits and an S-digit variant reads the first S.
//
// Scales.  Each proposal's kernel row is divided by a power of two s_q at
// or above max_r |B_r(x_q)| (Gaussian rows are at most 1, monomials of degree
// <= 3 at most max(1, max_d |x_d|)^3), each weight column by a power of two
// s_c above max_r |W_rc|.  Inside the unit ball s_q = 1, so the first digit
// spans the whole of [-127, 127].
//
// Products.  sum_r B_r W_rc = s_q s_c sum_l 254^-l D_l / 127^2 with
// D_l = sum_{i+j=l} sum_r a_i(r) b_j(r).  Every D_l with l < S is an exact
// int32 sum on the MFMA (at most 8 pairs * rows * 127^2 < 2^31 for
// rows <= 16384); the levels are combined once in FP64.  Dropping the pairs
// with i + j >= S and the digit remainders costs at most (S + 3) 254^-S of
// s_q s_c per kernel row.
//
// Tiles.  A workgroup of 4 waves (one per SIMD, so each wave may hold 512
// registers: the S level accumulators of two 32 x 32 blocks sit in AGPRs)
// computes 128 proposals x 64 columns; wave w computes proposals
// 32 w .. 32 w + 31 against all 64 columns with v_mfma_i32_32x32x32_i8,
// whose lane l holds A[l%32][16(l/32) + e] and B[16(l/32) + e][l%32] (e < 16,
// 16 int8 in 4 VGPRs) and accumulator element i = D[8(i/4) + 4(l/32) + i%4][l%32]
// (measured on gfx950).  Every wave loads its own operands straight from
// global memory into those registers (the four waves' B fragments coincide
// and are served by the CU's L1), one 32-row step ahead: no LDS, no
// barriers.  Against the LDS-staged 8-wave tile (two waves per SIMD, one
// barrier per 32-row step) this took 11-17% less time for S = 5..8 on the
// 3-detector shape; staging through LDS by direct global-to-LDS loads in a
// three- or four-stage ring was within 3% of it.  With any of these the
// kernel runs far below the matrix cores' own rate (the same MFMA sequence
// from registers alone reaches 0.88 of the int8 peak, from LDS alone 0.84):
// the digit traffic lowers the clock by about 18% under this load and
// stalls the rest.
//
// Memory layout of the digits (16-row groups g, G = rows / 16 of them):
//   rows   AS[i][g][q][16]   (q < nb, one chunk of proposals)
//   weights BS[j][g][c][16]  (c < Kp)
// so a workgroup's stage is one contiguous 1 KiB run per (digit, group).
#include "basis_rows.h"
#include "epilogue_setup.h"
#include "rbfl_internal.h"

namespace rbfl {

namespace {

constexpr int kMaxSlices = 8;
constexpr int kSplitQ = 128;     // proposals per workgroup (four waves of 32)
constexpr int kSplitC = 64;      // columns per workgroup (two 32-column blocks per wave)
constexpr int kSplitThreads = 256;
constexpr int kMaxSplitRows = 16384;

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

// Base-254 digits of v (|v| <= 1), packed one per byte.  No clamp is
// needed: |127 v| <= 127, and every remainder r has |r| <= 1/2 up to the
// FMA's rounding, so |254 r| rounds to at most 127.
template <int S>
__device__ __forceinline__ void digits(double v, int8_t out[S]) {
  double a = rint(v * 127.0);
  out[0] = (int8_t)a;
  double r = fma(v, 127.0, -a);
#pragma unroll
  for (int i = 1; i < S; ++i) {
    a = rint(r * 254.0);
    out[i] = (int8_t)a;
    r = fma(r, 254.0, -a);
  }
}

// The power-of-two row scale s_q >= max_r |B_r(x)| (see Scales above).  The
// bound m^3 is rounded as a monomial's own product is, so it also holds in
// floating point; a NaN coordinate leaves s_q = 1 (the epilogue flags it).
__device__ __forceinline__ double row_scale(const double x[4]) {
  double m = 1.0;
#pragma unroll
  for (int d = 0; d < 4; ++d) m = fmax(m, fabs(x[d]));
  int e = 0;
  const double f = frexp(m * m * m, &e);    // m^3 = f 2^e, f in [1/2, 1)
  return ldexp(1.0, f == 0.5 ? e - 1 : e);
}

__device__ __forceinline__ v4i pack16(const int8_t *b) {
  v4i v;
#pragma unroll
  for (int w = 0; w < 4; ++w)
    v[w] = (int)(uint8_t)b[4 * w] | ((int)(uint8_t)b[4 * w + 1] << 8) | ((int)(uint8_t)b[4 * w + 2] << 16) |
           ((int)(uint8_t)b[4 * w + 3] << 24);
  return v;
}

// The first S digits of the kernel rows of nb proposals and their row scales.
// Thread t = g * nb + q: proposal q, rows 16g .. 16g + 15.
template <int S>
__global__ void __launch_bounds__(256) k_split_rows(const EvalConsts *__restrict__ cp,
                                                    const double *__restrict__ params, int64_t ld, int64_t b0,
                                                    int64_t nb, const double *__restrict__ nodes,
                                                    v4i *__restrict__ AS, double *__restrict__ rscale) {
  const EvalConsts &c = *cp;
  const int G = c.rows / 16;
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= (int64_t)G * nb) return;
  const int g = (int)(t / nb);
  const int64_t q = t - (int64_t)g * nb;
  double x[4];
#pragma unroll
  for (int d = 0; d < 4; ++d) x[d] = params[d * ld + b0 + q] / c.semi[d];
  const int N = c.N, NM = c.N + c.M;
  const double sq = row_scale(x), inv = 1.0 / sq;    // powers of two: exact
  if (g == 0) rscale[q] = sq;
  int8_t dg[S][16];
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const int r = 16 * g + k;
    int8_t a[S];
    digits<S>(basis_row_fp64(r, N, NM, x, nodes + 4 * (int64_t)r, c.eps2, c.poly_idx) * inv, a);
#pragma unroll
    for (int i = 0; i < S; ++i) dg[i][k] = a[i];
  }
#pragma unroll
  for (int i = 0; i < S; ++i) AS[((int64_t)i * G + g) * nb + q] = pack16(dg[i]);
}

// Power-of-two scale of each weight column: 2^e > max_r |W[r][c]|.
__global__ void __launch_bounds__(256) k_col_scale(const double *__restrict__ W, int rows, int Kp,
                                                   double *__restrict__ scale) {
  const int col = blockIdx.x;
  __shared__ double red[256];
  double m = 0.0;
  for (int r = threadIdx.x; r < rows; r += 256) m = fmax(m, fabs(W[(int64_t)r * Kp + col]));
  red[threadIdx.x] = m;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    int e = 0;
    const double mx = red[0];
    if (mx > 0.0) frexp(mx, &e);
    scale[col] = mx > 0.0 ? ldexp(1.0, e) : 1.0;
  }
}

// All kMaxSlices digits of the scaled weights.  Thread t = g * Kp + col.
__global__ void __launch_bounds__(256) k_split_weights(const double *__restrict__ W, int rows, int Kp,
                                                       const double *__restrict__ scale, v4i *__restrict__ BS) {
  const int G = rows / 16;
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= (int64_t)G * Kp) return;
  const int g = (int)(t / Kp), col = (int)(t - (int64_t)g * Kp);
  const double inv = 1.0 / scale[col];    // a power of two: exact
  int8_t dg[kMaxSlices][16];
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    int8_t b[kMaxSlices];
    digits<kMaxSlices>(W[(int64_t)(16 * g + k) * Kp + col] * inv, b);
#pragma unroll
    for (int j = 0; j < kMaxSlices; ++j) dg[j][k] = b[j];
  }
#pragma unroll
  for (int j = 0; j < kMaxSlices; ++j) BS[((int64_t)j * G + g) * Kp + col] = pack16(dg[j]);
}

// Workgroups are dealt to the 8 XCDs in turn; this gives each XCD a
// contiguous range of logical tiles (a bijection for any grid size), so the
// column tiles of one proposal tile run on one XCD and share its L2.
__device__ __forceinline__ int64_t xcd_logical_block(int64_t b, int64_t nblk) {
  const int64_t x = b & 7, slot = b >> 3, base = nblk >> 3, extra = nblk & 7;
  return x * base + (x < extra ? x : extra) + slot;
}

// The level sums D_l of one tile, proposals q0 .. q0 + kSplitQ - 1 and
// columns c0 .. c0 + kSplitC - 1, over the digit pairs i + j < S: wave w
// holds acc[n][l] for proposals q0 + 32 w .. + 31 and columns c0 + 32 n ..
// + 31 (the 32 x 32 accumulator layout above).  Proposals past nb read the
// last proposal's digits.  Uses no LDS.
template <int S>
__device__ __forceinline__ void split_accumulate(const v4i *__restrict__ AS, int64_t nb, int rows,
                                                 const v4i *__restrict__ BS, int Kp, int64_t q0, int c0,
                                                 v16i (&acc)[2][S]) {
  const int lane = threadIdx.x & 63, wq = threadIdx.x >> 6;
  const int G = rows / 16, n_steps = rows / 32;
  const int kh = lane >> 5, ml = lane & 31;
  int64_t qa = q0 + wq * 32 + ml;
  qa = qa < nb ? qa : nb - 1;
  // per-lane byte offsets within a (digit, 16-row group) plane, added to
  // wave-uniform plane addresses
  const uint32_t oa = (uint32_t)(((int64_t)kh * nb + qa) * 16);
  const uint32_t ob = (uint32_t)(((int64_t)kh * Kp + c0 + ml) * 16);
  const char *ca = reinterpret_cast<const char *>(AS), *cb = reinterpret_cast<const char *>(BS);

#pragma unroll
  for (int n = 0; n < 2; ++n)
#pragma unroll
    for (int l = 0; l < S; ++l)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[n][l][r] = 0;
  // operands of one 32-row step: digit i of the wave's 32 proposals, digit j
  // of its two 32-column blocks; two register sets, the next step's in flight
  v4i a0[S], b0[2][S], a1[S], b1[2][S];
  auto load = [&](int st, v4i *a, v4i (*b)[S]) {
#pragma unroll
    for (int i = 0; i < S; ++i) {
      const char *pa = ca + ((int64_t)i * G + 2 * st) * nb * 16;
      const char *pb = cb + ((int64_t)i * G + 2 * st) * Kp * 16;
      a[i] = *reinterpret_cast<const v4i *>(pa + oa);
#pragma unroll
      for (int n = 0; n < 2; ++n) b[n][i] = *reinterpret_cast<const v4i *>(pb + ob + 512 * n);
    }
  };
  auto multiply = [&](const v4i *a, v4i (*b)[S]) {
#pragma unroll
    for (int i = 0; i < S; ++i)
#pragma unroll
      for (int j = 0; i + j < S; ++j)
#pragma unroll
        for (int n = 0; n < 2; ++n)
          acc[n][i + j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[i], b[n][j], acc[n][i + j], 0, 0, 0);
  };
  load(0, a0, b0);
  int st = 0;
  for (; st + 1 < n_steps; st += 2) {
    load(st + 1, a1, b1);
    multiply(a0, b0);
    if (st + 2 < n_steps) load(st + 2, a0, b0);
    multiply(a1, b1);
  }
  if (st < n_steps) multiply(a0, b0);     // an odd step count leaves the last step in set 0
}

// Output r of block n of a lane: sum_l 254^-l D_l (Horner from the highest
// level) scaled by s_c / 127^2 (sc) and s_q (rs).
template <int S>
__device__ __forceinline__ double split_value(const v16i (&acc)[2][S], int n, int r, double sc, double rs) {
  constexpr double kInv254 = 1.0 / 254.0;
  double y = (double)acc[n][S - 1][r];
#pragma unroll
  for (int l = S - 2; l >= 0; --l) y = fma(y, kInv254, (double)acc[n][l][r]);
  return y * sc * rs;
}

// One output tile Y[q][c] = s_q s_c sum_l 254^-l D_l[q][c] / 127^2: the tile
// of split_accumulate, stored for proposals below nb.
template <int S>
__device__ __forceinline__ void split_tile(const v4i *__restrict__ AS, int64_t nb, int rows,
                                           const v4i *__restrict__ BS, const double *__restrict__ cscale,
                                           const double *__restrict__ rscale, int Kp, double *__restrict__ Y,
                                           int64_t q0, int c0) {
  v16i acc[2][S];
  split_accumulate<S>(AS, nb, rows, BS, Kp, q0, c0, acc);
  const int lane = threadIdx.x & 63, wq = threadIdx.x >> 6;
  const int kh = lane >> 5, ml = lane & 31;
#pragma unroll
  for (int n = 0; n < 2; ++n) {
    const int col = c0 + 32 * n + ml;
    const double sc = cscale[col] * (1.0 / 16129.0);
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int64_t q = q0 + wq * 32 + 8 * (r >> 2) + 4 * kh + (r & 3);
      if (q >= nb) continue;
      Y[q * Kp + col] = split_value<S>(acc, n, r, sc, rscale[q]);
    }
  }
}

// One-dimensional grid over (proposal tile, column tile), the column tile
// fastest.
template <int S>
__global__ void __launch_bounds__(kSplitThreads, 1)
    k_split_contract(const v4i *__restrict__ AS, int64_t nb, int rows, const v4i *__restrict__ BS,
                     const double *__restrict__ cscale, const double *__restrict__ rscale, int Kp,
                     double *__restrict__ Y) {
  const int n_ct = Kp / kSplitC;
  const int64_t tile = xcd_logical_block(blockIdx.x, gridDim.x);
  split_tile<S>(AS, nb, rows, BS, cscale, rscale, Kp, Y, (tile / n_ct) * kSplitQ, (int)(tile % n_ct) * kSplitC);
}

// The split contraction that finishes ln L itself (frozen antenna
// patterns): the tile of split_accumulate, then each lane weights its 2 x 16
// outputs (the values split_tile would store) by their columns' ln L weights
// (lnl_weight), the 32 lanes of a row set add theirs (a fixed tree) and each
// wave writes one partial sum for each of its 32 proposals to
// part[column tile][proposal]; Y is never written.  Proposals outside the
// domain contribute 0 here (k_lnl_tiles writes their flag).
template <int S>
__global__ void __launch_bounds__(kSplitThreads, 1)
    k_split_lnl(const v4i *__restrict__ AS, int64_t nb, int rows, const v4i *__restrict__ BS,
                const double *__restrict__ cscale, const double *__restrict__ rscale, int Kp,
                const EvalConsts *__restrict__ cp, const EpiSetup *__restrict__ setups,
                const double2 *__restrict__ basis4, const int4 *__restrict__ coldesc, double *__restrict__ part,
                int64_t ldp) {
  const int n_ct = Kp / kSplitC;
  const int64_t tile = xcd_logical_block(blockIdx.x, gridDim.x);
  const int64_t q0 = (tile / n_ct) * kSplitQ;
  const int tc = (int)(tile % n_ct), c0 = tc * kSplitC;
  v16i acc[2][S];
  split_accumulate<S>(AS, nb, rows, BS, Kp, q0, c0, acc);
  const EvalConsts &c = *cp;
  const int lane = threadIdx.x & 63, wq = threadIdx.x >> 6;
  const int kh = lane >> 5, ml = lane & 31;
  int4 dsc[2];
  double sc[2];
#pragma unroll
  for (int n = 0; n < 2; ++n) {
    const int col = c0 + 32 * n + ml;
    dsc[n] = col < c.K ? coldesc[col] : make_int4(-1, 0, 0, 0);
    sc[n] = cscale[col] * (1.0 / 16129.0);
  }
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int64_t q = q0 + wq * 32 + 8 * (r >> 2) + 4 * kh + (r & 3);
    double sum = 0.0;
    if (q < nb && setups[q].status == 0) {
      const EpiSetup &o = setups[q];
      const double rs = rscale[q];
#pragma unroll
      for (int n = 0; n < 2; ++n) {
        if (dsc[n].x < 0) continue;
        sum = fma(lnl_weight(dsc[n], o, c.n_modes, c.T, c.q, basis4), split_value<S>(acc, n, r, sc[n], rs), sum);
      }
    }
#pragma unroll
    for (int m = 16; m >= 1; m >>= 1) sum += __shfl_xor(sum, m, 64);
    if (ml == 0 && q < nb) part[(int64_t)tc * ldp + q] = sum;
  }
}

// Multi-event batches: the first S digits (S = the event's) of the kernel
// rows of every event's proposals and their row scales, one launch.  Flat
// thread index t over the events (event e owns t0 .. t0 + (rows / 16) n - 1);
// within an event t - t0 = g n + q: proposal q, rows 16 g .. 16 g + 15.
__global__ void __launch_bounds__(256) k_ragged_split_rows(const EventDesc *__restrict__ ev, int n_ev,
                                                           int64_t total, const double *__restrict__ params,
                                                           int64_t ld) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= total) return;
  int lo = 0, hi = n_ev - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (ev[mid].t0 <= t) lo = mid;
    else hi = mid - 1;
  }
  const EventDesc &d = ev[lo];
  const EvalConsts &c = *d.consts;
  const int64_t local = t - d.t0;
  const int g = (int)(local / d.n);
  const int64_t q = local - (int64_t)g * d.n;
  double x[4];
#pragma unroll
  for (int dd = 0; dd < 4; ++dd) x[dd] = params[dd * ld + d.q0 + q] / c.semi[dd];
  const int N = c.N, NM = c.N + c.M;
  const double sq = row_scale(x), inv = 1.0 / sq;    // powers of two: exact
  if (g == 0) d.rscale[q] = sq;
  int8_t dg[kMaxSlices][16];
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const int r = 16 * g + k;
    int8_t a[kMaxSlices];
    digits<kMaxSlices>(basis_row_fp64(r, N, NM, x, d.nodes + 4 * (int64_t)r, c.eps2, c.poly_idx) * inv, a);
#pragma unroll
    for (int i = 0; i < kMaxSlices; ++i) dg[i][k] = a[i];
  }
  const int G = d.rows / 16;
  v4i *AS = static_cast<v4i *>(d.AS);
#pragma unroll
  for (int i = 0; i < kMaxSlices; ++i)
    if (i < d.S) AS[((int64_t)i * G + g) * d.n + q] = pack16(dg[i]);
}

// Multi-event batches: persistent split contraction over a work list of
// (event, proposal tile, column tile) items, every event of the list with S
// digits, column tile fastest within an event, events in decreasing cost;
// each workgroup takes the next item from an atomic counter until the list
// is exhausted (every workgroup reaches that exit).
template <int S>
__global__ void __launch_bounds__(kSplitThreads, 1)
    k_ragged_split_contract(const EventDesc *__restrict__ ev, int n_ev, int64_t total_items,
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
    split_tile<S>(static_cast<const v4i *>(d.AS), d.n, d.rows, static_cast<const v4i *>(d.BS), d.cscale, d.rscale,
                  d.Kp, d.Y, (local / d.tiles_c) * kSplitQ, (int)(local % d.tiles_c) * kSplitC);
  }
}

__global__ void k_zero_counters(unsigned long long *counter, int n) {
  if ((int)threadIdx.x < n) counter[threadIdx.x] = 0ull;
}

template <int S>
void launch_variant(const EvalConsts *c, const EvalConsts &hc, const double *params, int64_t ld, int64_t b0,
                    int64_t nb, const double *nodes, int8_t *AS, double *rscale, const int8_t *BS,
                    const double *cscale, double *Y, hipStream_t s, hipEvent_t mid) {
  static_assert(S <= kMaxSlices && kColTile % kSplitC == 0 && kRowChunk % 32 == 0,
                "K and the rows are padded to whole tiles");
  const int64_t G = hc.rows / 16;
  hipLaunchKernelGGL((k_split_rows<S>), dim3((unsigned)((G * nb + 255) / 256)), dim3(256), 0, s, c, params, ld, b0,
                     nb, nodes, reinterpret_cast<v4i *>(AS), rscale);
  RBFL_HIP(hipGetLastError());
  if (mid) RBFL_HIP(hipEventRecord(mid, s));
  const int64_t nblk = (nb + kSplitQ - 1) / kSplitQ * (hc.Kp / kSplitC);
  hipLaunchKernelGGL((k_split_contract<S>), dim3((unsigned)nblk), dim3(kSplitThreads), 0, s,
                     reinterpret_cast<const v4i *>(AS), nb, hc.rows, reinterpret_cast<const v4i *>(BS), cscale,
                     rscale, hc.Kp, Y);
  RBFL_HIP(hipGetLastError());
}

template <int S>
void launch_lnl_variant(const EvalConsts *c, const EvalConsts &hc, const double *params, int64_t ld, int64_t b0,
                        int64_t nb, const double *nodes, int8_t *AS, double *rscale, const int8_t *BS,
                        const double *cscale, const void *setups, const double2 *basis4, const int4 *coldesc,
                        double *part, int64_t ldp, hipStream_t s, hipEvent_t mid) {
  const int64_t G = hc.rows / 16;
  hipLaunchKernelGGL((k_split_rows<S>), dim3((unsigned)((G * nb + 255) / 256)), dim3(256), 0, s, c, params, ld, b0,
                     nb, nodes, reinterpret_cast<v4i *>(AS), rscale);
  RBFL_HIP(hipGetLastError());
  if (mid) RBFL_HIP(hipEventRecord(mid, s));
  const int64_t nblk = (nb + kSplitQ - 1) / kSplitQ * (hc.Kp / kSplitC);
  hipLaunchKernelGGL((k_split_lnl<S>), dim3((unsigned)nblk), dim3(kSplitThreads), 0, s,
                     reinterpret_cast<const v4i *>(AS), nb, hc.rows, reinterpret_cast<const v4i *>(BS), cscale,
                     rscale, hc.Kp, c, static_cast<const EpiSetup *>(setups), basis4, coldesc, part, ldp);
  RBFL_HIP(hipGetLastError());
}

}  // namespace

int split_ragged_tile_q() { return kSplitQ; }
int split_ragged_tile_c() { return kSplitC; }
int split_ragged_blocks_per_cu() { return 1; }

void launch_ragged_split_rows(const EventDesc *ev, int n_ev, int64_t total_threads, const double *params, int64_t ld,
                              hipStream_t s) {
  if (total_threads <= 0) return;
  hipLaunchKernelGGL(k_ragged_split_rows, dim3((unsigned)((total_threads + 255) / 256)), dim3(256), 0, s, ev, n_ev,
                     total_threads, params, ld);
  RBFL_HIP(hipGetLastError());
}

void launch_zero_counters(unsigned long long *counter, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_counters, dim3(1), dim3(64), 0, s, counter, n);
  RBFL_HIP(hipGetLastError());
}

void launch_ragged_split_contract(int S, const EventDesc *ev, int n_ev, int64_t total_items,
                                  unsigned long long *counter, int grid, hipStream_t s) {
  if (total_items <= 0) return;
  switch (S) {
    case 5: hipLaunchKernelGGL((k_ragged_split_contract<5>), dim3(grid), dim3(kSplitThreads), 0, s, ev, n_ev, total_items, counter); break;
    case 6: hipLaunchKernelGGL((k_ragged_split_contract<6>), dim3(grid), dim3(kSplitThreads), 0, s, ev, n_ev, total_items, counter); break;
    case 7: hipLaunchKernelGGL((k_ragged_split_contract<7>), dim3(grid), dim3(kSplitThreads), 0, s, ev, n_ev, total_items, counter); break;
    case 8: hipLaunchKernelGGL((k_ragged_split_contract<8>), dim3(grid), dim3(kSplitThreads), 0, s, ev, n_ev, total_items, counter); break;
    default: throw Error(RBFL_E_INVALID_ARG, "split form: digit count must be 5 .. 8");
  }
  RBFL_HIP(hipGetLastError());
}

int split_max_slices() { return kMaxSlices; }
int split_max_rows() { return kMaxSplitRows; }
int split_variant_count() { return 4; }
int split_variant_slices(int variant) { return 5 + variant; }

const char *split_variant_name(int v) {
  static const char *names[] = {"split s5 32x32x32", "split s6 32x32x32", "split s7 32x32x32", "split s8 32x32x32"};
  return names[v];
}

void launch_split_prepare(const double *W, int rows, int Kp, double *scale, int8_t *BS, hipStream_t s) {
  hipLaunchKernelGGL(k_col_scale, dim3(Kp), dim3(256), 0, s, W, rows, Kp, scale);
  RBFL_HIP(hipGetLastError());
  const int64_t n = (int64_t)(rows / 16) * Kp;
  hipLaunchKernelGGL(k_split_weights, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, W, rows, Kp, scale,
                     reinterpret_cast<v4i *>(BS));
  RBFL_HIP(hipGetLastError());
}

int split_col_tile() { return kSplitC; }

void launch_split_lnl(const EvalConsts *c, const EvalConsts &hc, const double *params, int64_t ld, int64_t b0,
                      int64_t nb, const double *nodes, int8_t *AS, double *rscale, const int8_t *BS,
                      const double *cscale, const void *setups, const double2 *basis4, const int4 *coldesc,
                      double *part, int64_t ldp, hipStream_t s, int variant, hipEvent_t mid) {
  if (hc.rows > kMaxSplitRows || hc.rows % 32 != 0 || hc.Kp % kSplitC != 0)
    throw Error(RBFL_E_UNSUPPORTED, "split form: rows must be a multiple of 32 and at most 16384");
  switch (variant) {
    case 0: launch_lnl_variant<5>(c, hc, params, ld, b0, nb, nodes, AS, rscale, BS, cscale, setups, basis4, coldesc, part, ldp, s, mid); break;
    case 1: launch_lnl_variant<6>(c, hc, params, ld, b0, nb, nodes, AS, rscale, BS, cscale, setups, basis4, coldesc, part, ldp, s, mid); break;
    case 2: launch_lnl_variant<7>(c, hc, params, ld, b0, nb, nodes, AS, rscale, BS, cscale, setups, basis4, coldesc, part, ldp, s, mid); break;
    case 3: launch_lnl_variant<8>(c, hc, params, ld, b0, nb, nodes, AS, rscale, BS, cscale, setups, basis4, coldesc, part, ldp, s, mid); break;
    default: throw Error(RBFL_E_INVALID_ARG, "unknown split-form variant");
  }
}

void launch_contract_split(const EvalConsts *c, const EvalConsts &hc, const double *params, int64_t ld, int64_t b0,
                           int64_t nb, const double *nodes, int8_t *AS, double *rscale, const int8_t *BS,
                           const double *cscale, double *Y, hipStream_t s, int variant, hipEvent_t mid) {
  if (hc.rows > kMaxSplitRows || hc.rows % 32 != 0 || hc.Kp % kSplitC != 0)
    throw Error(RBFL_E_UNSUPPORTED, "split form: rows must be a multiple of 32 and at most 16384");
  switch (variant) {
    case 0: launch_variant<5>(c, hc, params, ld, b0, nb, nodes, AS, rscale, BS, cscale, Y, s, mid); break;
    case 1: launch_variant<6>(c, hc, params, ld, b0, nb, nodes, AS, rscale, BS, cscale, Y, s, mid); break;
    case 2: launch_variant<7>(c, hc, params, ld, b0, nb, nodes, AS, rscale, BS, cscale, Y, s, mid); break;
    case 3: launch_variant<8>(c, hc, params, ld, b0, nb, nodes, AS, rscale, BS, cscale, Y, s, mid); break;
    default: throw Error(RBFL_E_INVALID_ARG, "unknown split-form variant");
  }
}

}  // namespace rbfl
