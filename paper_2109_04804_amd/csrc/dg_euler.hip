// Instantiation of the DGSEM operator kernels for the eps-scaled Euler equations (d = 2, 3).
#include "dg_launch.hpp"

hipError_t dg_launch_euler(const GeomHost& g, const LaunchReq& r, int f32) {
    if (g.D == 2) return launch_family<2, EulerEq<2>>(g, r, f32);
    if (g.D == 3) return launch_family<3, EulerEq<3>>(g, r, f32);
    return hipErrorInvalidValue;
}
