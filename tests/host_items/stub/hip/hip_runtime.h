/* Stand-in for <hip/hip_runtime.h> in the host build of the flash's
 * per-mixture work items: the function qualifiers become plain C++. */
#pragma once
#include "hip_runtime_api.h"
#include <cmath>
#define __device__
#define __host__
#define __global__
#define __forceinline__ inline __attribute__((always_inline))
using std::copysign;
using std::exp;
using std::fabs;
using std::fmax;
using std::fmin;
using std::isfinite;
using std::isnan;
using std::log;
using std::log1p;
using std::sqrt;
