// Shared device/host definitions of libmmp (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>
#include <mutex>
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

// Loads and stores of data that is read or written once per evaluation
// (the spectra of the y and z passes, B_d): marked non-temporal, so they do
// not displace from the caches what is read again soon (the kernel
// spectrum, the stage state).  The values are unchanged.
typedef float __attribute__((ext_vector_type(2))) nt_f2;
typedef float __attribute__((ext_vector_type(4))) nt_f4;
typedef double __attribute__((ext_vector_type(2))) nt_d2;
__device__ __forceinline__ float2 ntload(const float2* p) {
  const nt_f2 v = __builtin_nontemporal_load(reinterpret_cast<const nt_f2*>(p));
  return make_float2(v.x, v.y);
}
__device__ __forceinline__ double2 ntload(const double2* p) {
  const nt_d2 v = __builtin_nontemporal_load(reinterpret_cast<const nt_d2*>(p));
  return make_double2(v.x, v.y);
}
__device__ __forceinline__ float ntload(const float* p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ double ntload(const double* p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ void ntstore(float2* p, float2 v) {
  nt_f2 w;
  w.x = v.x; w.y = v.y;
  __builtin_nontemporal_store(w, reinterpret_cast<nt_f2*>(p));
}
__device__ __forceinline__ void ntstore(double2* p, double2 v) {
  nt_d2 w;
  w.x = v.x; w.y = v.y;
  __builtin_nontemporal_store(w, reinterpret_cast<nt_d2*>(p));
}
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

// ------------------------------------------------ embedded RK pairs --
// The five pairs of Table 2, as run on the device.  Stage s (1-based) of an
// attempt evaluates k_s at stage input s = y_n + h sum_{j<s} a[s-1][j] k_j;
// the input of the last stage ns is the propagated solution y_{n+1} (row
// ns-1 of a is b) and its slope becomes the next step's k_1.  For the pairs
// that are first-same-as-last that stage is their own; for the others it is
// the evaluation the next step would start with, so it is appended with
// c = 1, a = b and e = 0 and the number of evaluations per step is
// unchanged.  e = b - b* weighs the error estimate, q is its order.
// Coefficients: Heun; Bogacki & Shampine (1989); Cash & Karp (1990);
// Fehlberg (1969), 5th order propagated; Dormand & Prince (1980).
struct RKTab {
  int ns;
  int q;
  double c[7];
  double a[7][6];
  double e[7];
};

enum { RK_DP45 = 0, RK_HEUN = 1, RK_BS23 = 2, RK_CASHKARP = 3, RK_FEHLBERG = 4, RK_COUNT = 5 };

struct RK {
  static constexpr RKTab t[RK_COUNT] = {
      {7, 4,
       {0.0, 1.0 / 5, 3.0 / 10, 4.0 / 5, 8.0 / 9, 1.0, 1.0},
       {{0, 0, 0, 0, 0, 0},
        {1.0 / 5, 0, 0, 0, 0, 0},
        {3.0 / 40, 9.0 / 40, 0, 0, 0, 0},
        {44.0 / 45, -56.0 / 15, 32.0 / 9, 0, 0, 0},
        {19372.0 / 6561, -25360.0 / 2187, 64448.0 / 6561, -212.0 / 729, 0, 0},
        {9017.0 / 3168, -355.0 / 33, 46732.0 / 5247, 49.0 / 176, -5103.0 / 18656, 0},
        {35.0 / 384, 0.0, 500.0 / 1113, 125.0 / 192, -2187.0 / 6784, 11.0 / 84}},
       {71.0 / 57600, 0.0, -71.0 / 16695, 71.0 / 1920, -17253.0 / 339200, 22.0 / 525,
        -1.0 / 40}},
      {3, 1,
       {0.0, 1.0, 1.0, 0, 0, 0, 0},
       {{0, 0, 0, 0, 0, 0}, {1.0, 0, 0, 0, 0, 0}, {0.5, 0.5, 0, 0, 0, 0}},
       {-0.5, 0.5, 0, 0, 0, 0, 0}},
      {4, 2,
       {0.0, 1.0 / 2, 3.0 / 4, 1.0, 0, 0, 0},
       {{0, 0, 0, 0, 0, 0},
        {1.0 / 2, 0, 0, 0, 0, 0},
        {0.0, 3.0 / 4, 0, 0, 0, 0},
        {2.0 / 9, 1.0 / 3, 4.0 / 9, 0, 0, 0}},
       {-5.0 / 72, 1.0 / 12, 1.0 / 9, -1.0 / 8, 0, 0, 0}},
      {7, 4,
       {0.0, 1.0 / 5, 3.0 / 10, 3.0 / 5, 1.0, 7.0 / 8, 1.0},
       {{0, 0, 0, 0, 0, 0},
        {1.0 / 5, 0, 0, 0, 0, 0},
        {3.0 / 40, 9.0 / 40, 0, 0, 0, 0},
        {3.0 / 10, -9.0 / 10, 6.0 / 5, 0, 0, 0},
        {-11.0 / 54, 5.0 / 2, -70.0 / 27, 35.0 / 27, 0, 0},
        {1631.0 / 55296, 175.0 / 512, 575.0 / 13824, 44275.0 / 110592, 253.0 / 4096, 0},
        {37.0 / 378, 0.0, 250.0 / 621, 125.0 / 594, 0.0, 512.0 / 1771}},
       {-277.0 / 64512, 0.0, 6925.0 / 370944, -6925.0 / 202752, -277.0 / 14336, 277.0 / 7084,
        0.0}},
      {7, 4,
       {0.0, 1.0 / 4, 3.0 / 8, 12.0 / 13, 1.0, 1.0 / 2, 1.0},
       {{0, 0, 0, 0, 0, 0},
        {1.0 / 4, 0, 0, 0, 0, 0},
        {3.0 / 32, 9.0 / 32, 0, 0, 0, 0},
        {1932.0 / 2197, -7200.0 / 2197, 7296.0 / 2197, 0, 0, 0},
        {439.0 / 216, -8.0, 3680.0 / 513, -845.0 / 4104, 0, 0},
        {-8.0 / 27, 2.0, -3544.0 / 2565, 1859.0 / 4104, -11.0 / 40, 0},
        {16.0 / 135, 0.0, 6656.0 / 12825, 28561.0 / 56430, -9.0 / 50, 2.0 / 55}},
       {1.0 / 360, 0.0, -128.0 / 4275, -2197.0 / 75240, 1.0 / 50, 2.0 / 55, 0.0}},
  };
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
  // step-size rule: clip(safety (tol/err)^(1/(q+1)), fac_min, fac_max),
  // then at most dt_max (0: unbounded)
  double safety, fac_min, fac_max, dt_max;
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
  int ns;    // stages per attempt of the pair in use (RKTab::ns)
  int rk;    // index of that pair in RK::t
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

// A HIP graph capture on one thread must not overlap a call that
// synchronises the device (hipMalloc, hipFree, pinned host memory, stream
// creation and destruction) on another thread: such a call waits on the
// capturing stream and invalidates the capture.  The library takes this
// lock around every capture and every such call (the server's builder
// thread sets grids up while its worker thread captures and replays).
std::recursive_mutex& device_mutex();
using DeviceLock = std::lock_guard<std::recursive_mutex>;
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

// Pointers typed as global memory.  A kernel that reads its buffers through
// pointers loaded from a device-resident table would otherwise use flat
// memory instructions (the compiler cannot prove where such a pointer
// points): an aperture check on every access, and waits that cover LDS too.
template <typename T>
using gptr = __attribute__((address_space(1))) T*;
template <typename T>
using gcptr = const __attribute__((address_space(1))) T*;

// Input of RK stage s (1..ns): y_n, then sa/sb alternating, then y_new.
template <typename T>
__device__ __forceinline__ const T* stage_in(const Table<T>* tbl, int s) {
  if (s == 1) return tbl->yn;
  if (s == tbl->ns) return tbl->ynew;
  return (s & 1) ? tbl->sb : tbl->sa;
}
// Buffer the stage-s kernel writes the next stage's input into.
template <typename T>
__device__ __forceinline__ T* stage_out(const Table<T>* tbl, int s) {
  const int n = s + 1;
  if (n == tbl->ns) return tbl->ynew;
  return (n & 1) ? tbl->sb : tbl->sa;
}

__device__ __forceinline__ bool ctrl_stopped(const Ctrl* c) {
  return c != nullptr && (c->done != 0 || c->status != 0);
}

}  // namespace mmp
