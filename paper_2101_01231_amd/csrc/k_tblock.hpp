// Temporal blocking of the 2D composite constant-velocity step (k_tblock.hip).
#pragma once
#include <cstdint>

namespace ridg {

struct DevGeom;

constexpr int kTBlockSteps = 4;  // steps per launch

// 2D, theta = 1, 3, 6, 10 or 15 (orders 1-5), n[0] and n[1] multiples of 16.
bool tblock_shape_supported(int d, int ns, int n0, int n1);
// The composite taps: at most 9, spanning at most 3 elements in each direction.
bool tblock_taps_supported(const int32_t* taps, int ntaps);
// kTBlockSteps composite steps of `in` into `out` in one launch (in and out distinct).
int launch_tap_tblock(int ns, const DevGeom& g, const double* in, double* out, const double* A, const int32_t* taps,
                      int ntaps, void* stream);

}  // namespace ridg
