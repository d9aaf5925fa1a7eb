// Error reporting shared by the library's source files: the message of the
// last failure of each host thread, returned by acopf_last_error().
#pragma once

#include <hip/hip_runtime.h>

#include <string>

#include "acopf_admm.h"

namespace acopf {

std::string& last_error();  // per host thread

inline acopf_status fail(acopf_status s, const std::string& msg) {
  last_error() = msg;
  return s;
}

}  // namespace acopf

#define HIP_TRY(expr)                                                                          \
  do {                                                                                         \
    hipError_t _e = (expr);                                                                    \
    if (_e != hipSuccess)                                                                      \
      return ::acopf::fail(ACOPF_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(_e));  \
  } while (0)
