// Host-side error plumbing shared by the C ABI translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <stdexcept>
#include <string>

#include "../../include/flash.h"

namespace flash {

struct FlashError : std::runtime_error {
  flash_status st;
  FlashError(flash_status s, const std::string& m) : std::runtime_error(m), st(s) {}
};

// Records the thread-local error text read by flash_last_error and returns s.
flash_status record_error(flash_status s, const std::string& m);

}  // namespace flash

#define HIPCHK(x)                                                                                   \
  do {                                                                                              \
    hipError_t _e = (x);                                                                            \
    if (_e != hipSuccess)                                                                           \
      throw ::flash::FlashError(_e == hipErrorOutOfMemory ? FLASH_ERR_OUT_OF_MEMORY : FLASH_ERR_DEVICE, \
                                std::string(#x) + ": " + hipGetErrorString(_e));                    \
  } while (0)
