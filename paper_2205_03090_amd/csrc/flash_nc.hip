// flash_nc.hip -- the flash kernels for one component count, PTF_NC, set on
// the compiler command line (the build compiles this file once per nc so
// that the instantiations compile in parallel).
#include "flash_launch.hpp"

#ifndef PTF_NC
#error "PTF_NC must be defined"
#endif

namespace ptf {
template size_t nc_workspace_bytes<PTF_NC>(int64_t, int);
template int nc_flash<PTF_NC>(const FlashArgs &, const ptflash_problem *,
                              const ptflash_options *, void *, hipStream_t);
template int nc_backward<PTF_NC>(const BwdArgs &, const ptflash_problem *, hipStream_t);
template int nc_eval<PTF_NC>(int64_t, const double *, const double *, const double *,
                             const double *, const double *, const double *, const double *,
                             double *, double *, double *, hipStream_t);
}  // namespace ptf
