// tuned_gfx950.hpp -- launch shape of the persistent flash per component
// count on gfx950: lanes per mixture of the stability and of the split
// trust-region stage and of the two substitution stages (1: one mixture per
// lane; 16 or 32: one group of that many lanes per mixture) and threads per
// block, for a shared component set (row 0) and for one set per mixture
// (row 1).  Written by autotune.py from timed runs (the timings are in the
// autotune summary next to the profiles).
#pragma once

namespace ptf {

constexpr int kTunedLanesSa[2][21] = {{1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 32, 1, 32, 32, 32},
                                       {1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 32, 32, 32, 32, 32}};
constexpr int kTunedLanesSp[2][21] = {{1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 16, 32, 32, 32, 32},
                                       {1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 16, 16, 16, 32, 32, 32, 32, 32}};
constexpr int kTunedLanesSs[2][21] = {{1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1},
                                       {1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1}};
constexpr int kTunedBlock[2][21] = {{256, 256, 128, 128, 128, 128, 128, 128, 256, 256, 256, 64, 128, 128, 128, 128, 128, 128, 128, 256, 128},
                                     {256, 256, 64, 64, 64, 128, 64, 64, 128, 64, 256, 128, 256, 64, 64, 128, 128, 128, 128, 128, 64}};

constexpr int tuned_lanes_sa(int nc, bool pm)
{
    return (nc >= 0 && nc <= 20) ? kTunedLanesSa[pm ? 1 : 0][nc] : 1;
}

constexpr int tuned_lanes_sp(int nc, bool pm)
{
    return (nc >= 0 && nc <= 20) ? kTunedLanesSp[pm ? 1 : 0][nc] : 1;
}

constexpr int tuned_lanes_ss(int nc, bool pm)
{
    return (nc >= 0 && nc <= 20) ? kTunedLanesSs[pm ? 1 : 0][nc] : 1;
}

constexpr int tuned_block(int nc, bool pm)
{
    return (nc >= 0 && nc <= 20) ? kTunedBlock[pm ? 1 : 0][nc] : 256;
}

}  // namespace ptf
