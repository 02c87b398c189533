// Instantiation of the DGSEM operator kernels for linear advection (d = 1, 2, 3).
#include "dg_launch.hpp"

hipError_t dg_launch_advection(const GeomHost& g, const LaunchReq& r, int f32) {
    if (g.D == 1) return launch_family<1, AdvectionEq<1>>(g, r, f32);
    if (g.D == 2) return launch_family<2, AdvectionEq<2>>(g, r, f32);
    if (g.D == 3) return launch_family<3, AdvectionEq<3>>(g, r, f32);
    return hipErrorInvalidValue;
}
