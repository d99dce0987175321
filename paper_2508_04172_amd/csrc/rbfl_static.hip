// The FP64 online stage for callers that cannot allocate device memory: the
// same kernels as rbfl_eval's serial FP64 order (basis rows, MFMA
// contraction, epilogue, NaN count), with the basis rows and interpolated
// outputs of each chunk of proposals in a fixed device array compiled into
// the library instead of the handle's work space.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <string>

#include "rbfl_internal.h"

namespace rbfl {

namespace {

constexpr size_t kScratchBytes = RBFL_STATIC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;
constexpr int64_t kMinChunk = 64;

// One copy per GPU, held until the process ends.  In host code `scratch`
// names a host-side stand-in, never the device array: kernels and copies get
// the address that hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on `dev`, which must be the current device;
// looked up once per device.
void *scratch_on(int dev) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (dev < 0 || dev >= kMaxDevices) throw Error(RBFL_E_INVALID_ARG, "device index out of range");
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    RBFL_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) throw Error(RBFL_E_DEVICE, "hipGetSymbolAddress returned no address for the scratch array");
    g_scratch_ptr[dev] = p;
  }
  return g_scratch_ptr[dev];
}

// Proposals per chunk: each needs its basis rows (rows doubles, the chunk a
// multiple of 8 so that the rows' leading dimension is the chunk itself) and
// its outputs (Kp doubles).
int64_t static_chunk(const Ctx &c) {
  const size_t per = sizeof(double) * ((size_t)c.rows + (size_t)c.Kp);
  return (int64_t)(kScratchBytes / per) & ~int64_t(7);
}

void eval_static(Ctx &c, const double *params, int64_t n, double *lnl, hipStream_t s) {
  require(params != nullptr && lnl != nullptr, "params/lnl is NULL");
  require(n >= 0, "n must be >= 0");
  int dev = -1;
  RBFL_HIP(hipGetDevice(&dev));
  if (dev != c.device)
    throw Error(RBFL_E_INVALID_ARG, "the handle lives on device " + std::to_string(c.device) + ", device " +
                                        std::to_string(dev) + " is current");
  const int64_t chunk = static_chunk(c);
  if (chunk < kMinChunk)
    throw Error(RBFL_E_INVALID_ARG,
                "handle too large for the static work space: " + std::to_string(kMinChunk) + " proposals need " +
                    std::to_string(kMinChunk * 8 * ((int64_t)c.rows + c.Kp)) + " bytes, the array holds " +
                    std::to_string(kScratchBytes));
  double *Y = static_cast<double *>(scratch_on(dev));
  double *Bt = Y + (size_t)chunk * c.Kp;   // rows x rows_ld(nb) <= rows x chunk doubles
  const int v = c.variant[RBFL_FORM_FP64];
  for (int64_t b0 = 0; b0 < n; b0 += chunk) {
    const int64_t nb = std::min(chunk, n - b0);
    if (v < gemm_fp64_variants()) {
      launch_rows_fp64(c.consts.p, c.host_consts, params, n, b0, nb, c.nodes.p, Bt, s);
      launch_gemm_fp64(Bt, nb, c.host_consts, c.W.p, Y, s, v);
    } else {
      launch_contract_fp64(c.consts.p, c.host_consts, params, n, b0, nb, c.nodes.p, c.W.p, Y, s, 2);
    }
    launch_epilogue(c.consts.p, c.host_consts, params, n, b0, nb, Y, c.basis4.p, lnl, s);
  }
  launch_count_nan(lnl, n, c.nan_part.p, s);
}

}  // namespace

}  // namespace rbfl

extern "C" {

int32_t rbfl_eval_static(rbfl_handle h, const double *params, int64_t n, double *lnl, void *stream) {
  return rbfl::guarded([&] {
    rbfl::require(h != nullptr, "handle is NULL");
    rbfl::eval_static(h->c, params, n, lnl, reinterpret_cast<hipStream_t>(stream));
  });
}

}  // extern "C"
