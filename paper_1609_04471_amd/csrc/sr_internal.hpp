// sr_internal.hpp -- host functions shared by libsortrace's translation
// units.  Hidden: they are not part of the exported C ABI.
#pragma once

#include <stddef.h>

#include <string>

#include "sortrace.h"

namespace sr {

// Records `msg` as the calling thread's last error (sr_last_error_message)
// and returns `s`.
__attribute__((visibility("hidden"))) sr_status api_fail(sr_status s, const std::string& msg);
// Clears the calling thread's last error.
__attribute__((visibility("hidden"))) void api_clear_error();
// The argument checks every sort entry point applies to a key array: known
// dtype, non-NULL when n > 1, n below 2^36, aligned to the element size.
__attribute__((visibility("hidden"))) sr_status api_check_keys(sr_dtype dt, const void* keys, size_t n);

}  // namespace sr
