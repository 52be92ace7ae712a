// Rows of the harmonics of a template row: harmonic h of a signal at
// (r, z) sits at (h r, h z) (Section "Detailed explanation"), so the h-th
// harmonic of row j is the grid row nearest h z_j,
//   j_h = floor((h z_j - z_min) / z_step + 1/2),  z_j = z_min + j z_step,
// -1 when it falls off the grid (one template: row 0 kept when h z_0 = z_0).
// Each step is one IEEE double operation in the order written (no fused
// multiply-add), so every kernel takes exactly the rows of that definition.
#pragma once

#include <hip/hip_runtime.h>

namespace fdas {

__device__ __forceinline__ int harmonic_row(double z_min, double z_step, int n_z, int j, int h) {
#pragma clang fp contract(off)
    if (n_z == 1) return ((double)h * z_min == z_min) ? 0 : -1;
    const double t = z_min + (double)j * z_step;
    const double u = (double)h * t;
    const double v = u - z_min;
    const double x = v / z_step;
    const double f = floor(x + 0.5);
    if (!(f >= 0.0 && f < (double)n_z)) return -1;   // outside the grid (or NaN)
    return (int)f;
}

}  // namespace fdas
