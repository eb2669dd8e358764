// The 3D composite stencil, two z-neighbours per thread (k_stencil3d.hip).
#pragma once
#include <cstdint>

namespace ridg {

struct DevGeom;

// 3D, n[2] even, theta = 1, 4 or 10 (orders 1-3).
bool z2_supported(int d, int ns, int n2);
// One composite step of `in` into `out`, bitwise the one-element-per-thread composite kernel's result.
int launch_tap_z2(int ns, const DevGeom& g, const double* in, double* out, const double* A, const int32_t* taps,
                  int ntaps, void* stream);

}  // namespace ridg
