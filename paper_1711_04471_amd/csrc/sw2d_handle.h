// sw2d_handle.h - host-side access to a single-grid handle for the other C-ABI sources.
#pragma once

#include <hip/hip_runtime.h>

#include "sw2d.h"

namespace sw2d {
namespace detail {
// The stream and grid size of a single-grid handle (false for a null handle).
bool handle_info(sw2d_t h, hipStream_t* stream, int* nx, int* ny);
}  // namespace detail
}  // namespace sw2d
