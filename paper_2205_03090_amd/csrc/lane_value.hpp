// lane_value.hpp -- makes a wave-uniform value a per-lane (VGPR) value, so
// that the compiler does not keep it, or what it addresses, in scalar
// registers.
#pragma once

#include <stdint.h>

namespace ptf {

// The empty asm with a VGPR operand hides that every lane holds the same v.
__device__ __forceinline__ uintptr_t per_lane(uintptr_t v)
{
    __asm__ volatile("" : "+v"(v));
    return v;
}

}  // namespace ptf
