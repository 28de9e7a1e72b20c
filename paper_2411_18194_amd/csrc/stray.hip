// Stray field of the magnet in a layer of cells above it (paper: the
// out-of-plane stray field imaged at a height above a film, "Stray field
// imaging of the non-collinear antiferromagnet Mn3Sn"; the field itself is
// the magnetostatic field of "Magnetostatic field").
//
// B_t(x, y) = -mu0 sum_z sum_{x', y'} N(x - x', y - y', z_t - z) M(x', y', z),
// M = sum_s Ms_s m_s, with the cell-pair tensor table of stray_kernel_build.
// A direct tiled sum: a block owns 16x16 target cells and walks the source
// tiles of every layer, staging the 3x16x16 moments and the 6x31x31 tensor
// window of the tile pair in LDS; sums in FP64.  This is an output-time
// operation (one image per call), not part of a step.
#include <mutex>

#include "stray.h"

namespace mmp {

constexpr int kST = 16;               // tile edge
constexpr int kSW = 2 * kST - 1;      // offsets between two tiles

// The state is read through its slot in the grid's device pointer table
// (the controller swaps that table after accepted steps), so a launch needs
// no host read-back of the table.
template <typename T>
__global__ __launch_bounds__(256) void k_stray(const T* const* __restrict__ mslot, int nsub,
                                              double ms0, double ms1, double ms2,
                                              const double* __restrict__ k6, int nx, int ny,
                                              int nz, double* __restrict__ out) {
  const T* __restrict__ m = *mslot;
  __shared__ double sm[3][kST * kST];
  __shared__ double sk[6][kSW * kSW];
  const int tx = threadIdx.x % kST, ty = threadIdx.x / kST;
  const int x0 = blockIdx.x * kST, y0 = blockIdx.y * kST;
  const int xt = x0 + tx, yt = y0 + ty;
  const long N = (long)nx * ny * nz;
  const int wx = 2 * nx - 1, wy = 2 * ny - 1;
  const long ktot = (long)wx * wy * nz;
  double acc[3] = {0.0, 0.0, 0.0};
  const int ntx = (nx + kST - 1) / kST, nty = (ny + kST - 1) / kST;
  for (int z = 0; z < nz; ++z)
    for (int sty = 0; sty < nty; ++sty)
      for (int stx = 0; stx < ntx; ++stx) {
        const int sx0 = stx * kST, sy0 = sty * kST;
        __syncthreads();
        {
          // moments of the source tile (zero outside the grid)
          const int xs = sx0 + tx, ys = sy0 + ty;
          double v[3] = {0.0, 0.0, 0.0};
          if (xs < nx && ys < ny) {
            const long i = ((long)z * ny + ys) * nx + xs;
            for (int c = 0; c < 3; ++c) {
              v[c] = ms0 * (double)m[c * N + i];
              if (nsub >= 2) v[c] += ms1 * (double)m[3 * N + c * N + i];
              if (nsub == 3) v[c] += ms2 * (double)m[6 * N + c * N + i];
            }
          }
          for (int c = 0; c < 3; ++c) sm[c][threadIdx.x] = v[c];
        }
        // tensor window: offsets X = x0 - sx0 - 15 + ox, Y likewise
        for (int w = threadIdx.x; w < kSW * kSW; w += blockDim.x) {
          const int ox = w % kSW, oy = w / kSW;
          const int X = x0 - sx0 - (kST - 1) + ox, Y = y0 - sy0 - (kST - 1) + oy;
          const bool in = X > -nx && X < nx && Y > -ny && Y < ny;
          const long k = ((long)z * wy + (Y + ny - 1)) * wx + (X + nx - 1);
          for (int c = 0; c < 6; ++c) sk[c][w] = in ? k6[c * ktot + k] : 0.0;
        }
        __syncthreads();
        for (int j = 0; j < kST * kST; ++j) {
          const int sxl = j % kST, syl = j / kST;
          // offset (xt - xs, yt - ys) in window coordinates
          const int w = (ty - syl + kST - 1) * kSW + (tx - sxl + kST - 1);
          const double Mx = sm[0][j], My = sm[1][j], Mz = sm[2][j];
          const double nxx = sk[0][w], nyy = sk[1][w], nzz = sk[2][w];
          const double nxy = sk[3][w], nxz = sk[4][w], nyz = sk[5][w];
          acc[0] += nxx * Mx + nxy * My + nxz * Mz;
          acc[1] += nxy * Mx + nyy * My + nyz * Mz;
          acc[2] += nxz * Mx + nyz * My + nzz * Mz;
        }
      }
  if (xt < nx && yt < ny) {
    const long o = (long)yt * nx + xt;
    const long P = (long)nx * ny;
    for (int c = 0; c < 3; ++c) out[c * P + o] = -kMu0 * acc[c];
  }
}

template <typename T>
void launch_stray(const T* const* mslot, int nsub, double ms0, double ms1, double ms2,
                  const double* k6, int nx, int ny, int nz, double* out, hipStream_t st) {
  const dim3 g((nx + kST - 1) / kST, (ny + kST - 1) / kST);
  hipLaunchKernelGGL((k_stray<T>), g, dim3(kST * kST), 0, st, mslot, nsub, ms0, ms1, ms2, k6, nx,
                     ny, nz, out);
}

template void launch_stray<float>(const float* const*, int, double, double, double,
                                  const double*, int, int, int, double*, hipStream_t);
template void launch_stray<double>(const double* const*, int, double, double, double,
                                   const double*, int, int, int, double*, hipStream_t);

// ------------------------------------------------ fixed tensor table --
// Tensor table of the allocation-free stray-field call: one array per GPU,
// held for the life of the process.  Host code must not pass the array's
// name to a kernel (in host code it only names a host-side stand-in); the
// device address comes from hipGetSymbolAddress, taken once per device
// with that device current.
static __device__ __align__(256) double scratch[kStrayScratchDoubles];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

int stray_scratch(int dev, double** out) {
  *out = nullptr;
  if (dev < 0 || dev >= kMaxDevices) return -1;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) return -1;
    if (cur != dev && hipSetDevice(dev) != hipSuccess) return -1;
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (cur != dev) (void)hipSetDevice(cur);
    if (e != hipSuccess || !ptr) return -1;
    g_scratch_ptr[dev] = static_cast<double*>(ptr);
  }
  *out = g_scratch_ptr[dev];
  return 0;
}

}  // namespace mmp
