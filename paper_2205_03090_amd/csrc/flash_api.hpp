// flash_api.hpp -- what the C ABI (ptflash.hip) and the per-component-count
// translation units (flash_nc.hip, one object per nc) share: the argument
// blocks of the kernels and the per-nc launchers, which are defined in
// flash_launch.hpp and instantiated once per nc.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "ptflash.h"

namespace ptf {

constexpr int kMinNc = 2;
constexpr int kMaxNc = PTF_MAX_NC;

// Kernel arguments shared by every stage of the forward.
struct FlashArgs {
    int64_t n;
    const double *z, *T, *P;
    int max_pre_ss, max_ss, max_tr_sa, max_tr_split, max_polish, dem_every;
    int keep_factor;
    double tol_sa_ss, tol_sa_tr, tol_split_ss, tol_split_tr, tol_polish, eps_tm;
    int8_t *label;
    double *beta, *x, *y;
    int16_t *iters;
    uint16_t *status;
    uint32_t *flops;
    double *factor;
    double *tm;            // nullable: the value that decided stability
    int stability_only;    // stop after the stability decision (no split)
    const double *lnk0;    // nullable: initial ln K of the split substitutions
    const int8_t *hint;    // nullable: 0 known stable, 1 known unstable
};

// Arguments of the backward kernel.
struct BwdArgs {
    int64_t n;
    const double *z, *T, *P;
    const int8_t *label;
    const double *beta, *x, *y, *factor;
    const uint16_t *status;
    const double *gb, *gx, *gy;
    double *gz, *gT, *gP;
    double *gk;        // n*nc*nc (per mixture) or NULL when reduced
    double *kpart;     // npair*n contributions (pair-major) when reduced
};

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Per-nc launchers (flash_launch.hpp).  PM (props_per_mixture) selects the
// kernels that read one component set per mixture; the two layouts are
// instantiated in separate translation units.
template <int NC>
size_t nc_workspace_bytes(int64_t n, int form);
template <int NC, bool PM>
int nc_flash_pm(const FlashArgs &a, const ptflash_problem *p, const ptflash_options *o, void *ws,
                hipStream_t s);
template <int NC, bool PM>
int nc_backward_pm(const BwdArgs &b, const ptflash_problem *p, hipStream_t s);
template <int NC>
int nc_eval(int64_t n, const double *c, const double *T, const double *P, const double *Tc,
            const double *Pc, const double *om, const double *K, double *lnphi, double *Z,
            double *phi, hipStream_t s);

}  // namespace ptf
