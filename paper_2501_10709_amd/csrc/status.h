// Error reporting shared by the library's C entry points (the message is read by fm_last_error).
#pragma once

#include <hip/hip_runtime.h>

#include <string>

#include "../../include/finrl_mi.h"

namespace fm {

// Records msg as the calling thread's last error and returns s.
fm_status set_error(fm_status s, const std::string& msg);
// FM_OK for hipSuccess, else FM_ERR_DEVICE with "what: <HIP error string>".
fm_status device_error(hipError_t e, const char* what);

// Makes dev current for the scope (restores the previous device).
struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) == hipSuccess && prev != dev) (void)hipSetDevice(dev);
    else prev = -1;
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

}  // namespace fm
