// Shared device/host definitions of libmmp (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>
#include <string>

#include "mmp.h"

namespace mmp {

constexpr double kPi = 3.14159265358979323846;
constexpr double kMu0 = 4.0e-7 * kPi;        // exact 4 pi 1e-7 (T m/A)
constexpr double kMuB = 9.2740100783e-24;    // J/T
constexpr double kQe = 1.602176634e-19;      // C

// ------------------------------------------------------------ complex --
template <typename T> struct C2;
template <> struct C2<float> { using type = float2; };
template <> struct C2<double> { using type = double2; };
template <typename T> using cpx = typename C2<T>::type;

template <typename T>
__device__ __forceinline__ cpx<T> cmk(T re, T im) { cpx<T> r; r.x = re; r.y = im; return r; }
template <typename V>
__device__ __forceinline__ V cadd(V a, V b) { V r; r.x = a.x + b.x; r.y = a.y + b.y; return r; }
template <typename V>
__device__ __forceinline__ V csub(V a, V b) { V r; r.x = a.x - b.x; r.y = a.y - b.y; return r; }
template <typename V>
__device__ __forceinline__ V cmul(V a, V b) {
  V r; r.x = a.x * b.x - a.y * b.y; r.y = a.x * b.y + a.y * b.x; return r;
}
template <typename V>
__device__ __forceinline__ V cconj(V a) { V r; r.x = a.x; r.y = -a.y; return r; }
template <typename V, typename S>
__device__ __forceinline__ V cscale(V a, S s) { V r; r.x = a.x * s; r.y = a.y * s; return r; }

// ------------------------------------------------- Dormand-Prince 5(4) --
// Tableau of Dormand & Prince (1980); Table 2 of the paper lists the pair.
struct DP {
  static constexpr double c[7] = {0.0, 1.0 / 5, 3.0 / 10, 4.0 / 5, 8.0 / 9, 1.0, 1.0};
  static constexpr double a[7][6] = {
      {0, 0, 0, 0, 0, 0},
      {1.0 / 5, 0, 0, 0, 0, 0},
      {3.0 / 40, 9.0 / 40, 0, 0, 0, 0},
      {44.0 / 45, -56.0 / 15, 32.0 / 9, 0, 0, 0},
      {19372.0 / 6561, -25360.0 / 2187, 64448.0 / 6561, -212.0 / 729, 0, 0},
      {9017.0 / 3168, -355.0 / 33, 46732.0 / 5247, 49.0 / 176, -5103.0 / 18656, 0},
      {35.0 / 384, 0.0, 500.0 / 1113, 125.0 / 192, -2187.0 / 6784, 11.0 / 84},
  };
  // e = b(5th) - b*(4th)
  static constexpr double e[7] = {71.0 / 57600, 0.0, -71.0 / 16695, 71.0 / 1920,
                                  -17253.0 / 339200, 22.0 / 525, -1.0 / 40};
};

// ------------------------------------------------------- step control --
// Device-resident controller state: every kernel of a step reads h from
// here, so a whole run is enqueued without host round trips.
struct Ctrl {
  double t;          // accepted time
  double h;          // size of the step being attempted
  double dt;         // controller's proposal (unclipped)
  double t_end;      // end of the run segment
  double t_next;     // next output time (== t_end when not sampling)
  double sample_every;
  double t0;         // start of the run segment (sample times t0 + k*every)
  double tol;
  double dt_min;
  double err;        // last error estimate
  int64_t steps;
  int64_t rejects;
  int64_t max_attempts;
  int32_t land;      // h was clipped to land on t_next
  int32_t done;      // t reached t_end
  int32_t status;    // 0 or an MMP_E_* code
  int32_t fixed;     // fixed-step mode (accept always)
  int32_t sample_k;  // index of the next sample time
  int32_t nsamples;  // samples written
  int32_t sample_pending;
  int32_t accepted;  // last attempt accepted
  int32_t nonfinite; // set by kernels on NaN/Inf
  int32_t pad;
};

// Pointer table of one grid's integrator buffers (device resident so the
// controller can swap y_n/y_new and k1/k7 after an accepted step).
template <typename T>
struct Table {
  T* yn;     // accepted state  [nsub][3][N]
  T* ynew;   // stage-7 input = candidate y_{n+1}
  T* k[7];   // stage derivatives
  T* sa;     // stage inputs alternate between sa and sb
  T* sb;
  // elastic state (may be null): u, v and their stage derivatives
  T* un; T* unew; T* vn; T* vnew;
  T* ku[7]; T* kv[7];
  T* usa; T* usb; T* vsa; T* vsb;
};

// ------------------------------------------------------------ helpers --
inline int round_up(int v, int m) { return (v + m - 1) / m * m; }

// smallest 7-smooth even integer >= v (1 for v == 1)
inline int smooth_pad(int n) {
  if (n == 1) return 1;
  int v = 2 * n - 1;
  for (int p = v;; ++p) {
    if (p % 2) continue;
    int q = p;
    for (int f : {2, 3, 5, 7})
      while (q % f == 0) q /= f;
    if (q == 1) return p;
  }
}

// factor L into FFT radices (8 first, then 4, 2, 7, 5, 3)
inline int fft_radices(int L, int* out) {
  int n = 0;
  while (L % 8 == 0) { out[n++] = 8; L /= 8; }
  while (L % 4 == 0) { out[n++] = 4; L /= 4; }
  while (L % 2 == 0) { out[n++] = 2; L /= 2; }
  while (L % 7 == 0) { out[n++] = 7; L /= 7; }
  while (L % 5 == 0) { out[n++] = 5; L /= 5; }
  while (L % 3 == 0) { out[n++] = 3; L /= 3; }
  return L == 1 ? n : -1;
}

void set_error(const std::string& msg);
const char* get_error();

#define MMP_HIP_TRY(expr)                                                   \
  do {                                                                      \
    hipError_t e_ = (expr);                                                 \
    if (e_ != hipSuccess) {                                                 \
      ::mmp::set_error(std::string(#expr) + ": " + hipGetErrorString(e_)); \
      return MMP_E_HIP;                                                     \
    }                                                                       \
  } while (0)

// XCD-aware block remap: consecutive work items land on the same XCD (the
// hardware deals blocks round-robin over 8 XCDs), so neighbouring tiles
// share an L2.  nb_pad is the launched block count, a multiple of 8.
__device__ __forceinline__ int xcd_remap(int b, int nb_pad) {
  const int per = nb_pad >> 3;
  return (b & 7) * per + (b >> 3);
}

}  // namespace mmp

namespace mmp {

// Input of RK stage s (1..7): y_n, then sa/sb alternating, then y_new.
template <typename T>
__device__ __forceinline__ const T* stage_in(const Table<T>* tbl, int s) {
  if (s == 1) return tbl->yn;
  if (s == 7) return tbl->ynew;
  return (s & 1) ? tbl->sb : tbl->sa;
}
// Buffer the stage-s kernel writes the next stage's input into.
template <typename T>
__device__ __forceinline__ T* stage_out(const Table<T>* tbl, int s) {
  const int n = s + 1;
  if (n == 7) return tbl->ynew;
  return (n & 1) ? tbl->sb : tbl->sa;
}

__device__ __forceinline__ bool ctrl_stopped(const Ctrl* c) {
  return c != nullptr && (c->done != 0 || c->status != 0);
}

}  // namespace mmp
