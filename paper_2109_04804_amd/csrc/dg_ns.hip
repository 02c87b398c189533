// Instantiation of the DGSEM operator kernels for the Navier-Stokes equations with BR2 lifting
// (d = 2, 3; Sec. 5.1).
#include "dg_launch.hpp"

hipError_t dg_launch_ns(const GeomHost& g, const LaunchReq& r, int f32) {
    if (g.D == 2) return launch_family<2, NavierStokesEq<2>>(g, r, f32);
    if (g.D == 3) return launch_family<3, NavierStokesEq<3>>(g, r, f32);
    return hipErrorInvalidValue;
}
