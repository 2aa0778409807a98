// Boxcar injection that allocates nothing.
//
// nsfrb_inject_boxcars stages its host tables (cube pointers, records, sample
// offsets) in a device buffer it allocates and frees on every call. This
// variant stages them in a file-scope device array instead, so a caller that
// must not allocate (a serving loop that injects test pulses into live data,
// code that forbids hipMalloc) can still inject. Both run the same kernel.
//
// Each device holds its own copy of `scratch`; host code never passes the
// array's name to a kernel or a copy, only the device address that
// hipGetSymbolAddress returns for the current device (looked up once per
// device, on that device's first call).
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>
#include <string>

#include "../../include/nsfrb.h"
#include "host_util.h"
#include "nsfrb_internal.h"

namespace {

constexpr size_t kScratchBytes = (size_t)1 << 20;   // NSFRB_INJECT_STATIC_BYTES in nsfrb.h
constexpr int kMaxRecords = 4096;
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_scratch_dev[kMaxDevices];   // device address of `scratch`, per device

size_t align256(size_t n) { return (n + 255) & ~(size_t)255; }

// Device address of this device's copy of `scratch` (the current device).
nsfrb_status scratch_address(void** out) {
  int dev = -1;
  NSFRB_HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices)
    return nsfrb::host_fail(NSFRB_ERR_UNSUPPORTED, "device ordinal beyond the static-scratch table");
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    NSFRB_HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return nsfrb::host_fail(NSFRB_ERR_DEVICE, "hipGetSymbolAddress returned NULL for the scratch array");
    g_scratch_dev[dev] = p;
  }
  *out = g_scratch_dev[dev];
  return NSFRB_OK;
}

}  // namespace

extern "C" nsfrb_status nsfrb_inject_boxcars_static(void* const* d_cubes, int32_t n_cubes, int32_t dtype,
                                                    int32_t layout, int32_t n_pix, int32_t n_sub, int32_t n_time,
                                                    const nsfrb_boxcar* host_boxcars, const int32_t* host_offsets,
                                                    int32_t n, void* stream) {
  static_assert(sizeof(nsfrb_boxcar) == sizeof(nsfrb::BoxcarRec), "nsfrb_boxcar layout");
  nsfrb::host_clear_error();
  if (!d_cubes || n_cubes < 1 || !host_boxcars || !host_offsets || n < 1 || dtype < 0 || dtype > 2 ||
      (layout != 0 && layout != 1) || n_pix < 1 || n_sub < 1 || n_time < 1)
    return nsfrb::host_fail(NSFRB_ERR_INVALID_ARG, "bad injection arguments");
  if (n > kMaxRecords)
    return nsfrb::host_fail(NSFRB_ERR_INVALID_ARG, "more than 4096 boxcar records for the static scratch");
  const size_t bytes_ptr = align256(sizeof(void*) * (size_t)n_cubes);
  const size_t bytes_rec = align256(sizeof(nsfrb::BoxcarRec) * (size_t)n);
  const size_t bytes_off = sizeof(int32_t) * (size_t)n * (size_t)n_sub;
  if (bytes_ptr + bytes_rec + bytes_off > kScratchBytes)
    return nsfrb::host_fail(NSFRB_ERR_INVALID_ARG,
                            "tables need " + std::to_string(bytes_ptr + bytes_rec + bytes_off) +
                                " bytes, beyond the 1 MiB static scratch");
  for (int i = 0; i < n_cubes; ++i)
    if (!d_cubes[i]) return nsfrb::host_fail(NSFRB_ERR_INVALID_ARG, "cube pointer is NULL");
  for (int i = 0; i < n; ++i) {
    const nsfrb_boxcar& b = host_boxcars[i];
    if (b.cube < 0 || b.cube >= n_cubes || b.pixel < 0 || b.pixel >= n_pix || b.width < 1 || !std::isfinite(b.amp))
      return nsfrb::host_fail(NSFRB_ERR_INVALID_ARG, "boxcar record out of range");
    // pairwise check (no host allocation): records must name distinct (cube, pixel) pairs
    for (int j = 0; j < i; ++j)
      if (host_boxcars[j].cube == b.cube && host_boxcars[j].pixel == b.pixel)
        return nsfrb::host_fail(NSFRB_ERR_INVALID_ARG, "two boxcars share a (cube, pixel)");
  }
  void* base = nullptr;
  nsfrb_status st = scratch_address(&base);
  if (st != NSFRB_OK) return st;
  char* d_buf = static_cast<char*>(base);
  hipStream_t s = (hipStream_t)stream;
  // the copies are ordered on `stream` before the kernel that reads them, and
  // the call waits for the kernel, so the host tables may be released on return
  NSFRB_HIP_TRY(hipMemcpyAsync(d_buf, d_cubes, sizeof(void*) * (size_t)n_cubes, hipMemcpyHostToDevice, s));
  NSFRB_HIP_TRY(hipMemcpyAsync(d_buf + bytes_ptr, host_boxcars, sizeof(nsfrb::BoxcarRec) * (size_t)n,
                               hipMemcpyHostToDevice, s));
  NSFRB_HIP_TRY(hipMemcpyAsync(d_buf + bytes_ptr + bytes_rec, host_offsets, bytes_off, hipMemcpyHostToDevice, s));
  NSFRB_HIP_TRY(nsfrb::launch_inject_many((void* const*)d_buf, dtype, layout, n_pix, n_sub, n_time,
                                          (const nsfrb::BoxcarRec*)(d_buf + bytes_ptr),
                                          (const int*)(d_buf + bytes_ptr + bytes_rec), n, s));
  NSFRB_HIP_TRY(hipStreamSynchronize(s));
  return NSFRB_OK;
}
