// Surrogate training driver (rbfl_surrogate_train): training and held-out
// proposals drawn in the unit ball, the FP64 interpolant's outputs as
// targets, the optional FP64 least-squares polynomial base of the residual
// form, the MLP's training loop, and the held-out ln L check that decides
// whether the surrogate form uses the network.
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>

#include <algorithm>
#include <cmath>
#include <limits>
#include <string>
#include <vector>

#include "host_math.h"
#include "host_util.h"
#include "rbfl_internal.h"

namespace rbfl {

// Residual form of the surrogate: the least-squares polynomial of degree
// `degree` (all monomials, graded-lexicographic) in the training proposals'
// standardised coordinates u = (x - m) / s, x = delta_e / a, fitted to every
// output column in FP64 (normal equations P^T P B = P^T Y by FP64 products on
// the GPU, Cholesky on the host), kept in the handle, and subtracted from the
// targets Y [n][K] in place.
static void fit_surrogate_base(Ctx &c, const double *train_params, int64_t n, int degree, double *Y, hipStream_t s) {
  std::vector<double> xh((size_t)4 * n);
  RBFL_HIP(hipMemcpyAsync(xh.data(), train_params, sizeof(double) * 4 * n, hipMemcpyDeviceToHost, s));
  RBFL_HIP(hipStreamSynchronize(s));
  double m[4], sd[4];
  for (int d = 0; d < 4; ++d) {
    Sum a;
    for (int64_t i = 0; i < n; ++i) a.add(xh[(size_t)d * n + i] / c.semi[d]);
    m[d] = a.value() / (double)n;
    Sum v;
    for (int64_t i = 0; i < n; ++i) {
      const double e = xh[(size_t)d * n + i] / c.semi[d] - m[d];
      v.add(e * e);
    }
    sd[d] = sqrt(v.value() / (double)n);
    if (!(sd[d] > 0.0)) sd[d] = 1.0;
  }
  int poly[kMaxPoly][3];
  const int nb = monomials(degree, poly);
  std::vector<double> P((size_t)n * nb);
  for (int64_t i = 0; i < n; ++i) {
    double u[4];
    for (int d = 0; d < 4; ++d) u[d] = (xh[(size_t)d * n + i] / c.semi[d] - m[d]) / sd[d];
    for (int p = 0; p < nb; ++p) {
      double v = 1.0;
      for (int t = 0; t < 3; ++t)
        if (poly[p][t] >= 0) v *= u[poly[p][t]];
      P[(size_t)i * nb + p] = v;
    }
  }
  DevBuf<double> dP, dG, dR;
  dP.alloc(P.size());
  dG.alloc((size_t)nb * nb);
  dR.alloc((size_t)nb * c.K);
  RBFL_HIP(hipMemcpyAsync(dP.p, P.data(), sizeof(double) * P.size(), hipMemcpyHostToDevice, s));
  BlasHandle bh;
  blas_check(rocblas_set_stream(bh.h, s), "rocblas_set_stream");
  // column-major views: P^T is nb x n (ld nb), Y^T is K x n (ld K)
  const double one = 1.0, zero = 0.0, minus = -1.0;
  blas_check(rocblas_dgemm(bh.h, rocblas_operation_none, rocblas_operation_transpose, nb, nb, (int)n, &one, dP.p, nb,
                           dP.p, nb, &zero, dG.p, nb),
             "rocblas_dgemm (P^T P)");
  blas_check(rocblas_dgemm(bh.h, rocblas_operation_none, rocblas_operation_transpose, nb, c.K, (int)n, &one, dP.p, nb,
                           Y, c.K, &zero, dR.p, nb),
             "rocblas_dgemm (P^T Y)");
  std::vector<double> G((size_t)nb * nb), R((size_t)nb * c.K);
  RBFL_HIP(hipMemcpyAsync(G.data(), dG.p, sizeof(double) * G.size(), hipMemcpyDeviceToHost, s));
  RBFL_HIP(hipMemcpyAsync(R.data(), dR.p, sizeof(double) * R.size(), hipMemcpyDeviceToHost, s));
  RBFL_HIP(hipStreamSynchronize(s));
  // Cholesky G = L L^T (G symmetric positive definite for distinct proposals)
  std::vector<double> L((size_t)nb * nb, 0.0);
  for (int j = 0; j < nb; ++j) {
    double d = G[(size_t)j * nb + j];
    for (int k = 0; k < j; ++k) d -= L[(size_t)j * nb + k] * L[(size_t)j * nb + k];
    if (!(d > 0.0)) throw Error(RBFL_E_NUMERICAL, "surrogate base: the monomials of the training proposals are degenerate");
    L[(size_t)j * nb + j] = sqrt(d);
    for (int i = j + 1; i < nb; ++i) {
      double v = G[(size_t)i * nb + j];
      for (int k = 0; k < j; ++k) v -= L[(size_t)i * nb + k] * L[(size_t)j * nb + k];
      L[(size_t)i * nb + j] = v / L[(size_t)j * nb + j];
    }
  }
  // B [nb][K] row-major: column k solves G b = R[:, k]
  std::vector<double> B((size_t)nb * c.K), y(nb);
  for (int k = 0; k < c.K; ++k) {
    for (int i = 0; i < nb; ++i) {
      double v = R[(size_t)k * nb + i];
      for (int t = 0; t < i; ++t) v -= L[(size_t)i * nb + t] * y[t];
      y[i] = v / L[(size_t)i * nb + i];
    }
    for (int i = nb - 1; i >= 0; --i) {
      double v = y[i];
      for (int t = i + 1; t < nb; ++t) v -= L[(size_t)t * nb + i] * B[(size_t)t * c.K + k];
      B[(size_t)i * c.K + k] = v / L[(size_t)i * nb + i];
    }
  }
  c.sur_B.alloc(B.size());
  RBFL_HIP(hipMemcpyAsync(c.sur_B.p, B.data(), sizeof(double) * B.size(), hipMemcpyHostToDevice, s));
  // Y^T (K x n) -= B^T (K x nb, ld K) P^T (nb x n, ld nb)
  blas_check(rocblas_dgemm(bh.h, rocblas_operation_none, rocblas_operation_none, c.K, (int)n, nb, &minus, c.sur_B.p,
                           c.K, dP.p, nb, &one, Y, c.K),
             "rocblas_dgemm (Y - P B)");
  for (int d = 0; d < 4; ++d) {
    c.sur_ms[d] = m[d];
    c.sur_ms[4 + d] = sd[d];
  }
  c.sur_ms_d.alloc(8);
  RBFL_HIP(hipMemcpyAsync(c.sur_ms_d.p, c.sur_ms, sizeof(c.sur_ms), hipMemcpyHostToDevice, s));
  c.sur_poly.alloc(kMaxPoly * 3);
  RBFL_HIP(hipMemcpyAsync(c.sur_poly.p, poly, sizeof(poly), hipMemcpyHostToDevice, s));
  c.sur_U.alloc((size_t)c.cap * nb);
  RBFL_HIP(hipStreamSynchronize(s));
  c.sur_degree = degree;
  c.sur_nbase = nb;
}

void surrogate_train(Ctx &c, const rbfl_train_spec *sp, hipStream_t s) {
  if (c.graph_users > 0) throw Error(RBFL_E_STATE, "a sampler holds this handle's buffers: train before creating it");
  require(sp != nullptr, "spec is NULL");
  require(sp->hidden >= 8 && sp->hidden <= 1024, "hidden must be 8 .. 1024");
  require(sp->batch >= 1 && sp->batch <= 65536, "batch must be 1 .. 65536");
  require(sp->epochs >= 1, "epochs must be >= 1");
  require(sp->init_normals != nullptr && sp->train_params != nullptr, "NULL init or training proposals");
  require(sp->n_train >= sp->batch, "n_train must be >= batch");
  require(sp->n_holdout >= 0 && (sp->n_holdout == 0 || sp->holdout_params != nullptr), "held-out proposals");
  require(std::isfinite(sp->lr) && sp->lr > 0 && sp->beta1 >= 0 && sp->beta1 < 1 && sp->beta2 >= 0 &&
              sp->beta2 < 1 && sp->adam_eps > 0 && sp->threshold > 0,
          "Adam settings / threshold");
  require(sp->base_degree >= 0 && sp->base_degree <= 3, "base_degree must be 0 .. 3");
  const auto t0 = Clock::now();
  delete c.sur;
  c.sur = nullptr;
  c.sur_ok = false;
  c.sur = new Mlp();
  c.sur->init(4, sp->hidden, c.K, sp->init_normals);
  c.sur_degree = 0;
  c.sur_nbase = 0;
  c.sur_B.reset();
  c.sur_U.reset();
  if (c.cap == 0) reserve(c, 65536);
  c.sur_x.alloc((size_t)c.cap * 4);
  c.sur->reserve(std::max<int64_t>(c.cap, sp->batch));
  // targets: the FP64 interpolant at the training proposals (minus the
  // least-squares polynomial base in the residual form), standardised per column
  const int64_t n = sp->n_train;
  DevBuf<double> Ytr;
  Ytr.alloc((size_t)n * c.K);
  interp(c, sp->train_params, n, Ytr.p, RBFL_FORM_FP64, s);
  if (sp->base_degree > 0) fit_surrogate_base(c, sp->train_params, n, sp->base_degree, Ytr.p, s);
  c.sur_mu.alloc(c.K);
  c.sur_sd.alloc(c.K);
  launch_col_stats(Ytr.p, n, c.K, c.sur_mu.p, c.sur_sd.p, s);
  DevBuf<float> T, X;
  T.alloc((size_t)n * c.K);
  X.alloc((size_t)n * 4);
  launch_standardise(Ytr.p, n, c.K, c.sur_mu.p, c.sur_sd.p, T.p, s);
  launch_sur_inputs(sp->train_params, n, 0, n, c.consts.p, X.p, s);
  RBFL_HIP(hipStreamSynchronize(s));
  Ytr.reset();
  double first = 0.0, last = 0.0;
  const int64_t steps = n / sp->batch;
  for (int ep = 0; ep < sp->epochs; ++ep) {
    for (int64_t st = 0; st < steps; ++st) {
      const int64_t b0 = st * sp->batch;
      c.sur->loss_grad(X.p + b0 * 4, T.p + b0 * c.K, sp->batch, s);
      c.sur->adam(sp->lr, sp->beta1, sp->beta2, sp->adam_eps, s);
    }
    double l = 0.0;
    RBFL_HIP(hipMemcpyAsync(&l, c.sur->loss.p, sizeof(double), hipMemcpyDeviceToHost, s));
    RBFL_HIP(hipStreamSynchronize(s));
    if (ep == 0) first = l;
    last = l;
  }
  const double train_s = seconds_since(t0);
  // held-out check: ln L through the network against ln L through the interpolant
  double dmax = std::numeric_limits<double>::infinity(), dmed = dmax;
  bool accepted = false;
  if (sp->n_holdout > 0) {
    const int64_t m = sp->n_holdout;
    DevBuf<double> l_rbf, l_sur;
    l_rbf.alloc(m);
    l_sur.alloc(m);
    eval(c, sp->holdout_params, m, l_rbf.p, RBFL_FORM_FP64, s);
    c.sur_ok = true;
    eval(c, sp->holdout_params, m, l_sur.p, RBFL_FORM_SURROGATE, s);
    c.sur_ok = false;
    std::vector<double> a(m), b(m);
    RBFL_HIP(hipMemcpyAsync(a.data(), l_rbf.p, sizeof(double) * m, hipMemcpyDeviceToHost, s));
    RBFL_HIP(hipMemcpyAsync(b.data(), l_sur.p, sizeof(double) * m, hipMemcpyDeviceToHost, s));
    RBFL_HIP(hipStreamSynchronize(s));
    bool domains = true;
    std::vector<double> d;
    for (int64_t i = 0; i < m; ++i) {
      const bool fa = std::isfinite(a[i]), fb = std::isfinite(b[i]);
      if (fa != fb) domains = false;
      if (fa && fb) d.push_back(fabs(a[i] - b[i]));
    }
    if (!d.empty()) {
      std::sort(d.begin(), d.end());
      dmax = d.back();
      dmed = d[d.size() / 2];
    }
    accepted = domains && !d.empty() && dmax <= sp->threshold;
  }
  c.sur_ok = accepted;
  const double st[8] = {accepted ? 1.0 : 0.0, dmax, dmed, first, last, (double)sp->epochs, train_s, (double)n};
  for (int i = 0; i < 8; ++i) c.sur_stats[i] = st[i];
}

}  // namespace rbfl
