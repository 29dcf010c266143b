// Host-side helpers of the C ABI shared between its source files.
#pragma once
#include <hip/hip_runtime.h>

#include "ladl_kernels.hpp"
#include "ladlasso.h"

namespace ladl {

// record a message for ladl_last_error_detail() and return `code`
int host_fail(int code, const char *msg);
// LADL_EHIP with the HIP error text
int host_hipfail(hipError_t e, const char *what);
// LADL_OK or LADL_EINVAL with a message
int host_check_options(const ladl_options *o);
DevOpt host_dev_opt(const ladl_options &o);

} // namespace ladl
