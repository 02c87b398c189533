// Instantiation of the DGSEM operator kernels for viscous Burgers with BR1 lifting (d = 1, 2).
#include "dg_launch.hpp"

hipError_t dg_launch_burgers(const GeomHost& g, const LaunchReq& r, int f32) {
    if (g.D == 1) return launch_family<1, BurgersEq<1>>(g, r, f32);
    if (g.D == 2) return launch_family<2, BurgersEq<2>>(g, r, f32);
    return hipErrorInvalidValue;
}
