// Thread-local error text of the C ABI (bsm_last_error), shared by the ABI's source files.
#pragma once
#include <string>

#include "../../include/bsm.h"

namespace bsm {
// Records msg as the calling thread's last error and returns code.
bsm_status set_error(bsm_status code, const std::string& msg);
}  // namespace bsm
