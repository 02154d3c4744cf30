// Shared host-side helpers of libhlu: error reporting and HIP checks.
#pragma once
#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/hlu.h"

namespace hlu {

void set_error(const std::string& msg);
const char* get_error();

// An error with its status code, thrown inside the library and turned into
// a return code at the C boundary.
struct Error {
  hlu_status status;
  std::string msg;
};

[[noreturn]] inline void fail(hlu_status s, const std::string& m) { throw Error{s, m}; }

}  // namespace hlu

#define HLU_REQUIRE(cond, status, msg)                      \
  do {                                                      \
    if (!(cond)) ::hlu::fail((status), std::string(msg));   \
  } while (0)

#define HIP_OK(call)                                                               \
  do {                                                                             \
    hipError_t e_ = (call);                                                        \
    if (e_ != hipSuccess)                                                          \
      ::hlu::fail(HLU_ERR_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)
