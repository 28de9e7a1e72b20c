// Stray field of the magnet in a layer of cells above it.
#pragma once

#include "common.h"

namespace mmp {

// out[c][y][x] (3*nx*ny doubles, device) = -mu0 sum over the grid's cells of
// k6 (stray_kernel_build) times M = sum_s ms_s m_s (m: nsub*3*N, device).
template <typename T>
void launch_stray(const T* m, int nsub, double ms0, double ms1, double ms2, const double* k6,
                  int nx, int ny, int nz, double* out, hipStream_t st);

}  // namespace mmp
