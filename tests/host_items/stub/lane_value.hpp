// Host build: every value is the calling thread's own.
#pragma once
#include <stdint.h>
namespace ptf {
inline uintptr_t per_lane(uintptr_t v) { return v; }
}  // namespace ptf
