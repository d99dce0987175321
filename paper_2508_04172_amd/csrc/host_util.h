// Host helpers shared by the library's host files: rocBLAS status checks, a
// scoped rocBLAS handle and a wall-clock timer.
#pragma once

#include <rocblas/rocblas.h>

#include <chrono>
#include <string>

#include "rbfl_internal.h"

namespace rbfl {

inline void blas_check(rocblas_status s, const char *what) {
  if (s != rocblas_status_success)
    throw Error(s == rocblas_status_memory_error ? RBFL_E_OUT_OF_MEMORY : RBFL_E_DEVICE,
                std::string(what) + " failed with rocblas status " + std::to_string((int)s));
}

struct BlasHandle {
  rocblas_handle h = nullptr;
  BlasHandle() { blas_check(rocblas_create_handle(&h), "rocblas_create_handle"); }
  ~BlasHandle() {
    if (h) rocblas_destroy_handle(h);
  }
};

using Clock = std::chrono::steady_clock;
inline double seconds_since(Clock::time_point t) { return std::chrono::duration<double>(Clock::now() - t).count(); }

}  // namespace rbfl
