// host_util.h - error reporting and device allocation helpers of the host code.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdio>
#include <string>

#include "internal.h"

namespace aqmp {

void set_error(const std::string& msg);
void clear_error();
const char* last_error();

// Device allocation honouring the optional AQMP_MAX_DEVICE_BYTES cap; the
// cap is checked against the bytes this process has allocated through it.
int dev_alloc(void** p, size_t bytes);
void dev_free(void* p, size_t bytes);

#define AQMP_HIP(call)                                                          \
  do {                                                                          \
    hipError_t e_ = (call);                                                     \
    if (e_ != hipSuccess) {                                                     \
      ::aqmp::set_error(std::string(#call) + ": " + hipGetErrorString(e_));     \
      return AQMP_E_HIP;                                                        \
    }                                                                           \
  } while (0)

#define AQMP_FAIL(code, msg)        \
  do {                              \
    ::aqmp::set_error(msg);         \
    return (code);                  \
  } while (0)

}  // namespace aqmp
