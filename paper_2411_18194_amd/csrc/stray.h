// Stray field of the magnet in a layer of cells above it.
#pragma once

#include "common.h"

namespace mmp {

// out[c][y][x] (3*nx*ny doubles, device) = -mu0 sum over the grid's cells of
// k6 (stray_kernel_build) times M = sum_s ms_s m_s, with m (nsub*3*N,
// device) read on the device from *mslot (the state slot of the grid's
// pointer table).
template <typename T>
void launch_stray(const T* const* mslot, int nsub, double ms0, double ms1, double ms2,
                  const double* k6, int nx, int ny, int nz, double* out, hipStream_t st);

// Doubles in the per-device tensor table of the allocation-free stray-field
// call (16 MiB): grids with 6 nz (2nx - 1)(2ny - 1) up to this many.
constexpr long kStrayScratchDoubles = MMP_STRAY_NOALLOC_MAX;

// Device address of that table on device `dev` (looked up once per device,
// with `dev` made current for the lookup).  0 on success, -1 on a HIP error.
int stray_scratch(int dev, double** out);

}  // namespace mmp
