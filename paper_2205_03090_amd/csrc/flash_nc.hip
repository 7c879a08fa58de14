// flash_nc.hip -- the flash kernels for one component count, PTF_NC, and one
// layout of the component sets, PTF_PM (0: one set shared by the batch, 1:
// one set per mixture), both set on the compiler command line (the build
// compiles this file once per nc and layout so that the instantiations
// compile in parallel).
#include "flash_launch.hpp"

#ifndef PTF_NC
#error "PTF_NC must be defined"
#endif
#ifndef PTF_PM
#error "PTF_PM must be defined"
#endif

namespace ptf {
template int nc_flash_pm<PTF_NC, (PTF_PM != 0)>(const FlashArgs &, const ptflash_problem *,
                                                const ptflash_options *, void *, hipStream_t);
template int nc_backward_pm<PTF_NC, (PTF_PM != 0)>(const BwdArgs &, const ptflash_problem *,
                                                   hipStream_t);
#if PTF_PM == 0
template size_t nc_workspace_bytes<PTF_NC>(int64_t, int);
template int nc_eval<PTF_NC>(int64_t, const double *, const double *, const double *,
                             const double *, const double *, const double *, const double *,
                             double *, double *, double *, hipStream_t);
#endif
}  // namespace ptf
