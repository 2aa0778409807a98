// Host-side helpers shared by the library's translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <string>

#include "../../include/nsfrb.h"

namespace nsfrb {
// Record `msg` as this thread's last error and return `st`.
nsfrb_status host_fail(nsfrb_status st, const std::string& msg);
void host_clear_error();
}  // namespace nsfrb

#define NSFRB_HIP_TRY(expr)                                                                              \
  do {                                                                                                   \
    hipError_t e_ = (expr);                                                                              \
    if (e_ != hipSuccess)                                                                                \
      return ::nsfrb::host_fail(e_ == hipErrorOutOfMemory ? NSFRB_ERR_OUT_OF_MEMORY : NSFRB_ERR_DEVICE,  \
                                std::string(#expr) + ": " + hipGetErrorString(e_));                      \
  } while (0)
