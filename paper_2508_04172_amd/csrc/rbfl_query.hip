// Artefact and state export of a handle (rbfl_query): sizes, frame, nodes,
// weights, basis, node values, singular values, timings, kernel statistics,
// tuning state, the surrogate's parameters and base, NaN counts and time
// bands.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "rbfl_internal.h"

namespace rbfl {

static void copy_out(void *out, size_t bytes, const void *src, size_t need) {
  require(out != nullptr, "out is NULL");
  require(bytes >= need, "output buffer too small (need " + std::to_string(need) + " bytes)");
  std::memcpy(out, src, need);
}

void query(Ctx &c, int what, void *out, size_t bytes) {
  const int mn = std::min(c.N, c.T);
  switch (what) {
    case RBFL_Q_SIZES: {
      int64_t v[8] = {c.N, c.M, c.K, c.q, c.T, c.n_det, c.n_modes, c.half_w};
      copy_out(out, bytes, v, sizeof(v));
      return;
    }
    case RBFL_Q_FRAME: {
      double v[44];
      for (int i = 0; i < 4; ++i) v[i] = c.theta_c[i];
      for (int i = 0; i < 16; ++i) v[4 + i] = c.V[i];
      for (int i = 0; i < 4; ++i) v[20 + i] = c.lam[i];
      for (int i = 0; i < 4; ++i) v[24 + i] = c.semi[i];
      for (int i = 0; i < 16; ++i) v[28 + i] = c.metric[i];
      copy_out(out, bytes, v, sizeof(v));
      return;
    }
    case RBFL_Q_D_REF:
      copy_out(out, bytes, &c.d_ref, sizeof(double));
      return;
    case RBFL_Q_EPS:
      copy_out(out, bytes, &c.eps, sizeof(double));
      return;
    case RBFL_Q_BANDS: {
      // B, blocks, edges [B + 1], band times [B][n_modes]
      std::vector<double> v;
      v.push_back(c.n_bands);
      v.push_back(c.n_v);
      for (int64_t e : c.band_edges) v.push_back((double)e);
      for (int b = 0; b < c.n_bands; ++b)
        for (int a = 0; a < c.n_modes; ++a) v.push_back(c.host_consts.band_t[b][a]);
      copy_out(out, bytes, v.data(), sizeof(double) * v.size());
      return;
    }
    case RBFL_Q_F_REF:
      copy_out(out, bytes, &c.f_ref, sizeof(double));
      return;
    case RBFL_Q_SQUEEZE:
      copy_out(out, bytes, c.squeeze, sizeof(c.squeeze));
      return;
    case RBFL_Q_CENTRE: {
      double v[8];
      for (int i = 0; i < 6; ++i) v[i] = c.centre_opt[i];
      v[6] = c.centre_snr[0];
      v[7] = c.centre_snr[1];
      copy_out(out, bytes, v, sizeof(v));
      return;
    }
    case RBFL_Q_NODES:
      copy_out(out, bytes, c.x_nodes.data(), sizeof(double) * c.x_nodes.size());
      return;
    case RBFL_Q_NODE_PHYS:
      copy_out(out, bytes, c.phys_nodes.data(), sizeof(double) * c.phys_nodes.size());
      return;
    case RBFL_Q_NODE_VALUES:
      copy_out(out, bytes, c.node_values.data(), sizeof(double) * c.node_values.size());
      return;
    case RBFL_Q_SINGULAR:
      copy_out(out, bytes, c.singular.data(), sizeof(double) * c.singular.size());
      (void)mn;
      return;
    case RBFL_Q_COND:
      copy_out(out, bytes, &c.cond, sizeof(double));
      return;
    case RBFL_Q_TIMING:
      copy_out(out, bytes, c.timing, sizeof(c.timing));
      return;
    case RBFL_Q_WEIGHTS: {
      const size_t need = sizeof(double) * (size_t)(c.N + c.M) * c.K;
      require(out != nullptr && bytes >= need, "output buffer too small");
      RBFL_HIP(hipMemcpy2D(out, sizeof(double) * c.K, c.W.p, sizeof(double) * c.Kp, sizeof(double) * c.K, c.N + c.M,
                           hipMemcpyDeviceToHost));
      return;
    }
    case RBFL_Q_BASIS: {
      const size_t need = sizeof(double2) * c.basis.n;
      require(out != nullptr && bytes >= need, "output buffer too small");
      RBFL_HIP(hipMemcpy(out, c.basis.p, need, hipMemcpyDeviceToHost));
      return;
    }
    case RBFL_Q_Z_NODES: {
      const size_t need = sizeof(double2) * c.z_nodes.n;
      require(out != nullptr && bytes >= need, "output buffer too small");
      RBFL_HIP(hipMemcpy(out, c.z_nodes.p, need, hipMemcpyDeviceToHost));
      return;
    }
    case RBFL_Q_SURROGATE:
      copy_out(out, bytes, c.sur_stats, sizeof(c.sur_stats));
      return;
    case RBFL_Q_TUNE: {
      // per form: chosen variant, then 8 timings [ms] (0 = not timed)
      double v[4 * 9];
      for (int f = 0; f < 4; ++f) {
        v[9 * f] = c.variant[f];
        for (int i = 0; i < 8; ++i) v[9 * f + 1 + i] = c.tune_ms[f][i];
      }
      copy_out(out, bytes, v, sizeof(v));
      return;
    }
    case RBFL_Q_PIPELINE: {
      double v[7] = {(double)c.pipe, c.pipe_ms[0], c.pipe_ms[1], c.pipe_ms[2], c.pipe_ms[3],
                     c.lnl_gemm ? 1.0 : 0.0, c.lnl_gemm_ms};
      copy_out(out, bytes, v, sizeof(v));
      return;
    }
    case RBFL_Q_SPLIT_ERR:
      copy_out(out, bytes, c.split_err, sizeof(c.split_err));
      return;
    case RBFL_Q_SURROGATE_BASE: {
      if (!c.sur) throw Error(RBFL_E_STATE, "no surrogate trained on this handle");
      std::vector<double> v(10 + (size_t)c.sur_nbase * c.K, 0.0);
      v[0] = c.sur_degree;
      v[1] = c.sur_nbase;
      for (int i = 0; i < 8; ++i) v[2 + i] = c.sur_ms[i];
      if (c.sur_nbase) {
        RBFL_HIP(hipDeviceSynchronize());
        RBFL_HIP(hipMemcpy(v.data() + 10, c.sur_B.p, sizeof(double) * c.sur_nbase * c.K, hipMemcpyDeviceToHost));
      }
      copy_out(out, bytes, v.data(), sizeof(double) * v.size());
      return;
    }
    case RBFL_Q_SPLIT_STATE: {
      double v[3] = {c.split_tuned ? 1.0 : 0.0, c.split_ok ? 1.0 : 0.0,
                     (double)split_variant_slices(c.variant[RBFL_FORM_SPLIT])};
      copy_out(out, bytes, v, sizeof(v));
      return;
    }
    case RBFL_Q_SPLIT_ORDER: {
      double v[3] = {c.split_lnl ? 1.0 : 0.0, c.split_order_ms[0], c.split_order_ms[1]};
      copy_out(out, bytes, v, sizeof(v));
      return;
    }
    case RBFL_Q_NAN_COUNT: {
      require(out != nullptr && bytes >= sizeof(int64_t), "output buffer too small (need 8 bytes)");
      unsigned long long part[kNanParts];
      RBFL_HIP(hipDeviceSynchronize());
      RBFL_HIP(hipMemcpy(part, c.nan_part.p, sizeof(part), hipMemcpyDeviceToHost));
      int64_t total = 0;
      for (int i = 0; i < kNanParts; ++i) total += (int64_t)part[i];
      std::memcpy(out, &total, sizeof(total));
      return;
    }
    case RBFL_Q_SURROGATE_NET: {
      if (!c.sur) throw Error(RBFL_E_STATE, "no surrogate trained on this handle");
      const size_t np = (size_t)c.sur->np, need = sizeof(float) * (np + 2 * (size_t)c.K);
      require(out != nullptr, "out is NULL");
      require(bytes >= need, "output buffer too small (need " + std::to_string(need) + " bytes)");
      float *o = static_cast<float *>(out);
      RBFL_HIP(hipDeviceSynchronize());
      RBFL_HIP(hipMemcpy(o, c.sur->p.p, sizeof(float) * np, hipMemcpyDeviceToHost));
      RBFL_HIP(hipMemcpy(o + np, c.sur_mu.p, sizeof(float) * c.K, hipMemcpyDeviceToHost));
      RBFL_HIP(hipMemcpy(o + np + c.K, c.sur_sd.p, sizeof(float) * c.K, hipMemcpyDeviceToHost));
      return;
    }
    case RBFL_Q_KERNEL_STATS: {
      double v[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
      for (auto &t : c.timed) {
        RBFL_HIP(hipEventSynchronize(t.b));
        float ms = 0.0f;
        RBFL_HIP(hipEventElapsedTime(&ms, t.a, t.b));
        v[3 * t.kind] += ms;
        v[3 * t.kind + 1] += 1.0;
        v[3 * t.kind + 2] += (double)t.n;
      }
      c.drop_timed();
      copy_out(out, bytes, v, sizeof(v));
      return;
    }
    default:
      throw Error(RBFL_E_INVALID_ARG, "unknown query");
  }
}

}  // namespace rbfl
