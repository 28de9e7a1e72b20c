// Demagnetising field: zero-padded FFT convolution with the cell-averaged
// tensor (paper, Methods "Magnetostatic field"; the moment of a
// multi-sublattice cell is summed before the convolution).
//
// Pass structure (3-D grid):
//   x  forward  R2C of M (two real rows packed in one complex line), the
//               half spectrum stored transposed so y lines are contiguous
//   y  forward  zero-padded ny -> Py
//   z  fwd * K * inv  per (kx, ky) column, with the real octant kernel
//   y  inverse  Py -> crop ny
//   x  inverse  C2R (two rows per complex line), crop nx -> B_d
// A 2-D grid (nz == 1) fuses y forward, multiply and y inverse in one pass.
// Zero padding is never materialised in memory: the pads exist only in LDS.
#include "demag.h"
#include "demag4.h"

#include <vector>

namespace mmp {

// ------------------------------------------------------------- twiddles --
template <typename T>
__global__ void k_twiddles(cpx<T>* tw, int L) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= L) return;
  double s, c;
  sincospi(-2.0 * (double)j / (double)L, &s, &c);
  tw[j] = cmk<T>((T)c, (T)s);
}

template <typename T>
void build_twiddles(cpx<T>* tw, int L, hipStream_t st) {
  hipLaunchKernelGGL(k_twiddles<T>, dim3((L + 255) / 256), dim3(256), 0, st, tw, L);
}
template void build_twiddles<float>(cpx<float>*, int, hipStream_t);
template void build_twiddles<double>(cpx<double>*, int, hipStream_t);

// --------------------------------------------------------------- x pass --
template <typename T>
struct XArgs {
  const Table<T>* tbl;
  const Ctrl* ctrl;
  int stage;
  T ms0, ms1, ms2;
  int nsub;
  cpx<T>* S1;
  T* Bd;
  const cpx<T>* tw;
  int nx, ny, nz, Px, Hx, ldy, ty;
  Rad rad;
};

// The pass bodies take the block's coordinates (and the stage) as
// arguments: the single-grid kernels pass blockIdx, the batched kernels
// the entry of their work table.
template <typename T, bool P2, bool TWL>
__device__ __forceinline__ void fftx_fwd_body(const XArgs<T>& a, int stage, int bx, int by,
                                              int bz) {
  using V = cpx<T>;
  if (ctrl_stopped(a.ctrl)) return;
  extern __shared__ char smem_raw[];
  V* buf = reinterpret_cast<V*>(smem_raw);
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int c = bz, z = by, y0 = bx * a.ty;
  const int nl = a.ty >> 1;
  const long N = (long)a.nx * a.ny * a.nz;
  const gcptr<T> m = (gcptr<T>)stage_in(a.tbl, stage);
  const gcptr<T> m0 = m + (long)c * N + (long)z * a.ny * a.nx;
  const gcptr<T> m1 = m0 + 3 * N;
  for (int idx = tid; idx < nl * a.Px; idx += nthr) {
    const int q = idx / a.Px, x = idx - q * a.Px;
    const int ya = y0 + 2 * q, yb = ya + 1;
    T re = 0, im = 0;
    if (x < a.nx) {
      if (ya < a.ny) {
        re = a.ms0 * m0[(long)ya * a.nx + x];
        if (a.nsub >= 2) re += a.ms1 * m1[(long)ya * a.nx + x];
        if (a.nsub == 3) re += a.ms2 * m1[3 * N + (long)ya * a.nx + x];
      }
      if (yb < a.ny) {
        im = a.ms0 * m0[(long)yb * a.nx + x];
        if (a.nsub >= 2) im += a.ms1 * m1[(long)yb * a.nx + x];
        if (a.nsub == 3) im += a.ms2 * m1[3 * N + (long)yb * a.nx + x];
      }
    }
    buf[q * a.Px + x] = cmk<T>(re, im);
  }
  const V* tw = a.tw;
  if constexpr (TWL) {
    // the twiddle table in LDS beside the lines: every stage reads it there
    V* twl = buf + (nl * a.Px);
    for (int i = tid; i < a.Px; i += nthr) twl[i] = a.tw[i];
    tw = twl;
  }
  __syncthreads();
  lds_fft<T, false, P2>(buf, tw, a.Px, nl, a.Px, a.rad.n, a.rad.code, tid, nthr);
  // unpack the two real spectra and store them transposed
  V* out = a.S1 + ((long)(c * a.nz + z) * a.Hx) * a.ldy + y0;
  for (int idx = tid; idx < nl * a.Hx; idx += nthr) {
    const int q = idx % nl, kx = idx / nl;
    const V zk = buf[q * a.Px + kx];
    const int km = kx == 0 ? 0 : a.Px - kx;
    const V zm = buf[q * a.Px + km];
    const T h = T(0.5);
    V xa = cmk<T>(h * (zk.x + zm.x), h * (zk.y - zm.y));
    V xb = cmk<T>(h * (zk.y + zm.y), h * (zm.x - zk.x));
    V* o = out + (long)kx * a.ldy + 2 * q;
    o[0] = xa;
    o[1] = xb;
  }
}

template <typename T, bool P2, bool TWL>
__global__ void k_fftx_fwd(XArgs<T> a) {
  fftx_fwd_body<T, P2, TWL>(a, a.stage, blockIdx.x, blockIdx.y, blockIdx.z);
}

template <typename T, bool P2, bool TWL>
__device__ __forceinline__ void fftx_inv_body(const XArgs<T>& a, int bx, int by, int bz) {
  using V = cpx<T>;
  if (ctrl_stopped(a.ctrl)) return;
  extern __shared__ char smem_raw[];
  V* buf = reinterpret_cast<V*>(smem_raw);
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int c = bz, z = by, y0 = bx * a.ty;
  const int nl = a.ty >> 1;
  const V* in = a.S1 + ((long)(c * a.nz + z) * a.Hx) * a.ldy + y0;
  for (int idx = tid; idx < nl * a.Hx; idx += nthr) {
    const int q = idx % nl, kx = idx / nl;
    const V* ip = in + (long)kx * a.ldy + 2 * q;
    const V xa = ip[0], xb = ip[1];
    buf[q * a.Px + kx] = cmk<T>(xa.x - xb.y, xa.y + xb.x);
    if (kx > 0 && 2 * kx < a.Px)
      buf[q * a.Px + a.Px - kx] = cmk<T>(xa.x + xb.y, xb.x - xa.y);
  }
  const V* tw = a.tw;
  if constexpr (TWL) {
    // the twiddle table in LDS beside the lines: every stage reads it there
    V* twl = buf + (nl * a.Px);
    for (int i = tid; i < a.Px; i += nthr) twl[i] = a.tw[i];
    tw = twl;
  }
  __syncthreads();
  lds_fft<T, true, P2>(buf, tw, a.Px, nl, a.Px, a.rad.n, a.rad.code, tid, nthr);
  const long N = (long)a.nx * a.ny * a.nz;
  T* out = a.Bd + (long)c * N + (long)z * a.ny * a.nx;
  for (int idx = tid; idx < nl * a.nx; idx += nthr) {
    const int q = idx / a.nx, x = idx - q * a.nx;
    const int ya = y0 + 2 * q;
    const V v = buf[q * a.Px + x];
    if (ya < a.ny) out[(long)ya * a.nx + x] = v.x;
    if (ya + 1 < a.ny) out[(long)(ya + 1) * a.nx + x] = v.y;
  }
}

template <typename T, bool P2, bool TWL>
__global__ void k_fftx_inv(XArgs<T> a) {
  fftx_inv_body<T, P2, TWL>(a, blockIdx.x, blockIdx.y, blockIdx.z);
}

// --------------------------------------------------------------- y pass --
template <typename T>
struct YArgs {
  const Ctrl* ctrl;
  const cpx<T>* in;
  cpx<T>* out;
  const cpx<T>* tw;
  int nlines, nvalid_in, ld_in, nvalid_out, ld_out, L, nl;
  Rad rad;
};

template <typename T, bool INV, bool P2, bool TWL>
__device__ __forceinline__ void ffty_body(const YArgs<T>& a, int bx) {
  using V = cpx<T>;
  if (ctrl_stopped(a.ctrl)) return;
  extern __shared__ char smem_raw[];
  V* buf = reinterpret_cast<V*>(smem_raw);
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int l0 = bx * a.nl;
  for (int idx = tid; idx < a.nl * a.L; idx += nthr) {
    const int q = idx / a.L, e = idx - q * a.L;
    const int gl = l0 + q;
    V v = cmk<T>(0, 0);
    if (gl < a.nlines && e < a.nvalid_in) v = a.in[(long)gl * a.ld_in + e];
    buf[q * a.L + e] = v;
  }
  const V* tw = a.tw;
  if constexpr (TWL) {
    // the twiddle table in LDS beside the lines: every stage reads it there
    V* twl = buf + (a.nl * a.L);
    for (int i = tid; i < a.L; i += nthr) twl[i] = a.tw[i];
    tw = twl;
  }
  __syncthreads();
  lds_fft<T, INV, P2>(buf, tw, a.L, a.nl, a.L, a.rad.n, a.rad.code, tid, nthr);
  for (int idx = tid; idx < a.nl * a.nvalid_out; idx += nthr) {
    const int q = idx / a.nvalid_out, e = idx - q * a.nvalid_out;
    const int gl = l0 + q;
    if (gl < a.nlines) a.out[(long)gl * a.ld_out + e] = buf[q * a.L + e];
  }
}

template <typename T, bool INV, bool P2, bool TWL>
__global__ void k_ffty(YArgs<T> a) {
  ffty_body<T, INV, P2, TWL>(a, blockIdx.x);
}

// Symmetric 3x3 multiply with the octant kernel; sy/sz flip the odd parts.
template <typename T>
__device__ __forceinline__ void kmul(cpx<T>& mx, cpx<T>& my, cpx<T>& mz, const T* __restrict__ K,
                                     long kidx, long kstride, T sy, T sz, bool three_d) {
  const T kxx = K[kidx], kyy = K[kidx + kstride], kzz = K[kidx + 2 * kstride];
  const T kxy = sy * K[kidx + 3 * kstride];
  T kxz = 0, kyz = 0;
  if (three_d) {
    kxz = sz * K[kidx + 4 * kstride];
    kyz = sy * sz * K[kidx + 5 * kstride];
  }
  const cpx<T> bx = cmk<T>(kxx * mx.x + kxy * my.x + kxz * mz.x, kxx * mx.y + kxy * my.y + kxz * mz.y);
  const cpx<T> by = cmk<T>(kxy * mx.x + kyy * my.x + kyz * mz.x, kxy * mx.y + kyy * my.y + kyz * mz.y);
  const cpx<T> bz = cmk<T>(kxz * mx.x + kyz * my.x + kzz * mz.x, kxz * mx.y + kyz * my.y + kzz * mz.y);
  mx = bx;
  my = by;
  mz = bz;
}

// 2-D grids: y forward, multiply, y inverse for nk kx columns x 3 components.
template <typename T>
struct M2Args {
  const Ctrl* ctrl;
  cpx<T>* S1;     // [3][1][Hx][ldy]
  const T* K;     // [6][1][Hx][Hy]
  const cpx<T>* tw;
  int ny, Py, Hx, Hy, ldy, nk;
  Rad rad;
};

template <typename T, bool P2, bool TWL>
__device__ __forceinline__ void ffty_mul2d_body(const M2Args<T>& a, int bx) {
  using V = cpx<T>;
  if (ctrl_stopped(a.ctrl)) return;
  extern __shared__ char smem_raw[];
  V* buf = reinterpret_cast<V*>(smem_raw);
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int kx0 = bx * a.nk;
  const int L = a.Py;
  const int nl = 3 * a.nk;
  for (int idx = tid; idx < nl * L; idx += nthr) {
    const int line = idx / L, e = idx - line * L;
    const int c = line / a.nk, j = line - c * a.nk;
    const int kx = kx0 + j;
    V v = cmk<T>(0, 0);
    if (kx < a.Hx && e < a.ny) v = a.S1[((long)c * a.Hx + kx) * a.ldy + e];
    buf[line * L + e] = v;
  }
  const V* tw = a.tw;
  if constexpr (TWL) {
    // the twiddle table in LDS beside the lines: every stage reads it there
    V* twl = buf + (nl * L);
    for (int i = tid; i < L; i += nthr) twl[i] = a.tw[i];
    tw = twl;
  }
  __syncthreads();
  lds_fft<T, false, P2>(buf, tw, L, nl, L, a.rad.n, a.rad.code, tid, nthr);
  const long kstride = (long)a.Hx * a.Hy;
  for (int idx = tid; idx < a.nk * L; idx += nthr) {
    const int j = idx / L, ky = idx - j * L;
    const int kx = kx0 + j;
    if (kx >= a.Hx) continue;
    const int kyo = ky <= L / 2 ? ky : L - ky;
    const T sy = ky <= L / 2 ? T(1) : T(-1);
    V mx = buf[(0 * a.nk + j) * L + ky];
    V my = buf[(1 * a.nk + j) * L + ky];
    V mz = buf[(2 * a.nk + j) * L + ky];
    kmul<T>(mx, my, mz, a.K, (long)kx * a.Hy + kyo, kstride, sy, T(1), false);
    buf[(0 * a.nk + j) * L + ky] = mx;
    buf[(1 * a.nk + j) * L + ky] = my;
    buf[(2 * a.nk + j) * L + ky] = mz;
  }
  __syncthreads();
  lds_fft<T, true, P2>(buf, tw, L, nl, L, a.rad.n, a.rad.code, tid, nthr);
  for (int idx = tid; idx < nl * a.ny; idx += nthr) {
    const int line = idx / a.ny, e = idx - line * a.ny;
    const int c = line / a.nk, j = line - c * a.nk;
    const int kx = kx0 + j;
    if (kx < a.Hx) a.S1[((long)c * a.Hx + kx) * a.ldy + e] = buf[line * L + e];
  }
}

template <typename T, bool P2, bool TWL>
__global__ void k_ffty_mul2d(M2Args<T> a) {
  ffty_mul2d_body<T, P2, TWL>(a, blockIdx.x);
}

// 3-D grids: z forward, multiply, z inverse for tk ky values of one kx.
template <typename T>
struct ZArgs {
  const Ctrl* ctrl;
  cpx<T>* S2;     // [3][nz][Hx][Py]
  const T* K;     // [6][Hz][Hx][Hy]
  const cpx<T>* tw;
  int nz, Pz, Hx, Py, Hy, Hz, tk, ls;
  Rad rad;
};

template <typename T, bool P2, bool TWL>
__device__ __forceinline__ void fftz_mul_body(const ZArgs<T>& a, int bx, int by) {
  using V = cpx<T>;
  if (ctrl_stopped(a.ctrl)) return;
  extern __shared__ char smem_raw[];
  V* buf = reinterpret_cast<V*>(smem_raw);
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int kx = by, ky0 = bx * a.tk;
  const int L = a.Pz;
  const int nl = 3 * a.tk;
  const long zstride = (long)a.Hx * a.Py;
  const long cstride = (long)a.nz * zstride;
  const V* base = a.S2 + (long)kx * a.Py + ky0;
  for (int idx = tid; idx < nl * L; idx += nthr) {
    const int j = idx % a.tk;
    const int r = idx / a.tk;
    const int z = r % L, c = r / L;
    V v = cmk<T>(0, 0);
    if (z < a.nz && ky0 + j < a.Py) v = base[c * cstride + z * zstride + j];
    buf[(c * a.tk + j) * a.ls + z] = v;
  }
  const V* tw = a.tw;
  if constexpr (TWL) {
    // the twiddle table in LDS beside the lines: every stage reads it there
    V* twl = buf + (nl * a.ls);
    for (int i = tid; i < L; i += nthr) twl[i] = a.tw[i];
    tw = twl;
  }
  __syncthreads();
  lds_fft<T, false, P2>(buf, tw, L, nl, a.ls, a.rad.n, a.rad.code, tid, nthr);
  const long kstride = (long)a.Hz * a.Hx * a.Hy;
  for (int idx = tid; idx < a.tk * L; idx += nthr) {
    const int j = idx % a.tk, kz = idx / a.tk;
    const int ky = ky0 + j;
    if (ky >= a.Py) continue;
    const int kyo = ky <= a.Py / 2 ? ky : a.Py - ky;
    const T sy = ky <= a.Py / 2 ? T(1) : T(-1);
    const int kzo = kz <= L / 2 ? kz : L - kz;
    const T sz = kz <= L / 2 ? T(1) : T(-1);
    V mx = buf[(0 * a.tk + j) * a.ls + kz];
    V my = buf[(1 * a.tk + j) * a.ls + kz];
    V mz = buf[(2 * a.tk + j) * a.ls + kz];
    kmul<T>(mx, my, mz, a.K, ((long)kzo * a.Hx + kx) * a.Hy + kyo, kstride, sy, sz, true);
    buf[(0 * a.tk + j) * a.ls + kz] = mx;
    buf[(1 * a.tk + j) * a.ls + kz] = my;
    buf[(2 * a.tk + j) * a.ls + kz] = mz;
  }
  __syncthreads();
  lds_fft<T, true, P2>(buf, tw, L, nl, a.ls, a.rad.n, a.rad.code, tid, nthr);
  V* obase = a.S2 + (long)kx * a.Py + ky0;
  for (int idx = tid; idx < 3 * a.tk * a.nz; idx += nthr) {
    const int j = idx % a.tk;
    const int r = idx / a.tk;
    const int z = r % a.nz, c = r / a.nz;
    if (ky0 + j < a.Py) obase[c * cstride + z * zstride + j] = buf[(c * a.tk + j) * a.ls + z];
  }
}

template <typename T, bool P2, bool TWL>
__global__ void k_fftz_mul(ZArgs<T> a) {
  fftz_mul_body<T, P2, TWL>(a, blockIdx.x, blockIdx.y);
}

// --------------------------------------------------------- batched passes --
// One launch of a pass for many grids: block b runs the pass body of grid
// work[b].x at block coordinates (work[b].y, .z, .w) with that grid's
// arguments.  256 threads per block; the dynamic LDS is the largest any
// grid's block needs.
constexpr int kMultiThreads = 256;

template <typename T>
__global__ __launch_bounds__(kMultiThreads) void k_fftx_fwd_multi(
    const XArgs<T>* __restrict__ args, const int4* __restrict__ work, int stage) {
  const int4 w = work[blockIdx.x];
  fftx_fwd_body<T, false, true>(args[w.x], stage, w.y, w.z, w.w);
}

template <typename T>
__global__ __launch_bounds__(kMultiThreads) void k_fftx_inv_multi(
    const XArgs<T>* __restrict__ args, const int4* __restrict__ work) {
  const int4 w = work[blockIdx.x];
  fftx_inv_body<T, false, true>(args[w.x], w.y, w.z, w.w);
}

template <typename T, bool INV>
__global__ __launch_bounds__(kMultiThreads) void k_ffty_multi(const YArgs<T>* __restrict__ args,
                                                              const int4* __restrict__ work) {
  const int4 w = work[blockIdx.x];
  ffty_body<T, INV, false, true>(args[w.x], w.y);
}

template <typename T>
__global__ __launch_bounds__(kMultiThreads) void k_fftz_mul_multi(
    const ZArgs<T>* __restrict__ args, const int4* __restrict__ work) {
  const int4 w = work[blockIdx.x];
  fftz_mul_body<T, false, true>(args[w.x], w.y, w.z);
}

template <typename T>
__global__ __launch_bounds__(kMultiThreads) void k_ffty_mul2d_multi(
    const M2Args<T>* __restrict__ args, const int4* __restrict__ work) {
  const int4 w = work[blockIdx.x];
  ffty_mul2d_body<T, false, true>(args[w.x], w.y);
}

// ------------------------------------------------------------------ plan --
constexpr long kMixedTarget = 2048;
constexpr size_t kLdsMax = 65536;   // dynamic LDS of one block


static int threads_for(long elems) {
  long t = (elems + kMaxE - 1) / kMaxE;
  t = (t + 63) / 64 * 64;
  if (t < 64) t = 64;
  return (int)t;
}

// complex elements one block may hold in LDS (64 KiB)
static long lds_cap(int real_bytes) { return 65536 / (2 * real_bytes); }

// An open axis is zero-padded to P >= 2n - 1; a periodic one is cyclic
// with P = n.  P is 1 or even and 7-smooth, at most 4096.
static bool pad_ok(int n, int P, bool periodic = false) {
  if (n == 1) return P == 1;
  if (periodic ? P != n : P < 2 * n - 1) return false;
  if ((P & 1) || P > 4096) return false;
  int r[16];
  const int nr = fft_radices(P, r);
  return nr >= 0 && nr <= 15;
}

// threads and LDS bytes of each pass for the plan's shapes
static int x_threads(const DemagPlan& p, int ty) {
  return p.p2x ? (ty / 2) * split_l2(p.Px) : threads_for((long)(ty / 2) * p.Px);
}
static int y_threads(const DemagPlan& p, int nl) {
  return p.p2y ? nl * split_l2(p.Py) : threads_for((long)nl * p.Py);
}
static int m2_threads(const DemagPlan& p) {
  return p.p2y ? 3 * p.nk * split_l2(p.Py) : threads_for((long)3 * p.nk * p.Py);
}
static int z_threads(const DemagPlan& p) { return threads_for((long)3 * p.tk * p.Pz); }

static bool pow2_in(int v, int lo, int hi) { return v >= lo && v <= hi && is_pow2(v); }

int demag_plan_check(const DemagPlan& p, int real_bytes) {
  const long cap = lds_cap(real_bytes);
  for (int ty : {p.tyf, p.tyi}) {
    if (!pow2_in(ty, 2, 16) || (long)(ty / 2) * p.Px > cap) return -1;
    if (x_threads(p, ty) > (p.p2x ? 256 : 1024)) return -1;
  }
  if (p.nz == 1) {
    if (!pow2_in(p.nk, 1, 64) || (long)3 * p.nk * p.Py > cap) return -1;
    if (m2_threads(p) > (p.p2y ? 256 : 1024)) return -1;
  } else {
    for (int nl : {p.nlyf, p.nlyi}) {
      if (!pow2_in(nl, 1, 64) || (long)nl * p.Py > cap) return -1;
      if (y_threads(p, nl) > (p.p2y ? 256 : 1024)) return -1;
    }
    if (p.p2z) {
      if (!zreg_waves_ok(real_bytes, p.Pz, p.zq, p.zw)) return -1;
      if (p.zt != 64 && p.zt != 128 && p.zt != 256) return -1;
      if (p.zmode < 0 || p.zmode > 1) return -1;
      if (p.zmode == 1 &&
          (real_bytes != 4 || p.zw != 1 || zk_lds_bytes(p.Pz, p.zq, p.zt) > (long)kLdsMax))
        return -1;
    } else {
      if (!pow2_in(p.tk, 1, 64) || (long)3 * p.tk * (p.Pz + 1) > cap) return -1;
      if (z_threads(p) > 1024) return -1;
    }
  }
  return 0;
}

int demag_plan(int nx, int ny, int nz, int real_bytes, const int* pads, DemagPlan* p,
               const int* rep) {
  DemagPlan d;
  d.nx = nx; d.ny = ny; d.nz = nz;
  if (rep)
    for (int a = 0; a < 3; ++a) d.rep[a] = rep[a];
  if (d.rep[2] != 0) return -1;
  const bool px = d.rep[0] > 0, py = d.rep[1] > 0;
  if (pads) {
    if (!pad_ok(nx, pads[0], px) || !pad_ok(ny, pads[1], py) || !pad_ok(nz, pads[2])) return -1;
    d.Px = pads[0]; d.Py = pads[1]; d.Pz = pads[2];
  } else {
    d.Px = px ? nx : smooth_pad(nx);
    d.Py = py ? ny : smooth_pad(ny);
    d.Pz = smooth_pad(nz);
    if (!pad_ok(nx, d.Px, px) || !pad_ok(ny, d.Py, py) || !pad_ok(nz, d.Pz)) return -1;
  }
  d.Hx = d.Px / 2 + 1; d.Hy = d.Py / 2 + 1; d.Hz = d.Pz / 2 + 1;
  int rr[3][16];
  d.rx = make_rad(rr[0], fft_radices(d.Px, rr[0]));
  d.ry = make_rad(rr[1], fft_radices(d.Py, rr[1]));
  d.rz = make_rad(rr[2], fft_radices(d.Pz, rr[2]));
  // power-of-two axes: register four-step kernels (FP64 lines up to 2048
  // points); the register z pass spreads a column over zq lanes
  const int lmax = real_bytes == 8 ? 2048 : 4096;
  d.p2x = is_pow2(d.Px) && d.Px <= lmax;
  d.p2y = is_pow2(d.Py) && d.Py <= lmax;
  d.p2z = is_pow2(d.Pz) && d.Pz <= 64;
  d.ldy = round_up(ny, 16);
  const long cap = lds_cap(real_bytes);
  // the mixed-radix LDS passes are latency-bound: at most kMixedTarget
  // complex elements per block, so that even small grids launch many
  // blocks (the power-of-two register passes take as many as fit)
  const long mcap = std::min<long>(cap, kMixedTarget);
  // x passes: the most rows per block that the LDS, the block size and the
  // grid (no more rows than it has) allow
  int ty = 2;
  const long xcap = d.p2x ? cap : mcap;
  while (ty < 16 && (long)ty * d.Px <= xcap && ty < ny + (ny & 1)) ty *= 2;
  while (ty > 2 && ((long)(ty / 2) * d.Px > cap || x_threads(d, ty) > (d.p2x ? 256 : 1024)))
    ty /= 2;
  d.tyf = d.tyi = ty;
  // y passes: lines per block
  {
    int n = 1;
    if (d.p2y) {
      const int l2 = split_l2(d.Py);
      while (n < 64 && (long)(2 * n) * d.Py <= cap && 2 * n * l2 <= 256) n *= 2;
    } else {
      while (n < 8 && (long)(2 * n) * d.Py <= mcap) n *= 2;
    }
    d.nlyf = d.nlyi = n;
  }
  // 2-D fused pass: kx columns per block
  {
    int k = 1;
    if (d.p2y) {
      const int l2 = split_l2(d.Py);
      while (k < 64 && (long)3 * (2 * k) * d.Py <= cap && 3 * (2 * k) * l2 <= 256) k *= 2;
    } else {
      while (k < 64 && (long)3 * (2 * k) * d.Py <= mcap) k *= 2;
    }
    d.nk = k;
  }
  // z pass: mixed-radix ky per block; register lanes per column
  {
    int tk = 64;
    while (tk > 1 && (long)3 * tk * (d.Pz + 1) > mcap) tk /= 2;
    d.tk = tk;
    // FP32 columns of up to 32 points: one lane per column, two waves per
    // SIMD (the column's 192 registers and the transform's temporaries fit
    // the 256 of a wave); otherwise the fewest lanes whose share of a
    // column takes at most 96 registers, one wave's worth of the rest
    int q = 1, w = 1;
    if (real_bytes == 4 && zreg_waves_ok(real_bytes, d.Pz, 1, 2)) {
      w = 2;
    } else {
      while (q < 4 &&
             (!zreg_ok(real_bytes, d.Pz, q) || zreg_data_vgprs(real_bytes, d.Pz, q) > 96))
        q *= 2;
      if (!zreg_ok(real_bytes, d.Pz, q)) q = 1;
    }
    d.zq = q;
    d.zw = w;
    d.zt = 128;
    if (d.p2z && !zreg_ok(real_bytes, d.Pz, d.zq)) d.p2z = false;
  }
  d.s1_elems = (size_t)3 * nz * d.Hx * d.ldy;
  d.s2_elems = nz > 1 ? (size_t)3 * nz * d.Hx * d.Py : 0;
  d.k_elems = (size_t)6 * d.Hz * d.Hx * d.Hy;
  if (demag_plan_check(d, real_bytes) != 0) return -1;
  *p = d;
  return 0;
}

// --------------------------------------------------------------- passes --
template <typename T>
void demag_pass(int pass, const DemagPlan& p, const DemagBufs<T>& b, const Table<T>* tbl,
                int stage, const Ctrl* ctrl, T ms0, T ms1, int nsub, hipStream_t st, T ms2) {
  using V = cpx<T>;
  switch (pass) {
    case DP_XF:
    case DP_XI: {
      const bool inv = pass == DP_XI;
      const int ty = inv ? p.tyi : p.tyf;
      const dim3 g((p.ny + ty - 1) / ty, p.nz, 3);
      const size_t lds = (size_t)(ty / 2) * p.Px * sizeof(V);
      if (p.p2x) {
        const size_t lds4 = x4_lds_bytes(p.Px, ty / 2, inv, (int)sizeof(V));
        X4Args<T> a;
        a.tbl = tbl; a.ctrl = ctrl; a.stage = stage; a.ms0 = ms0; a.ms1 = ms1; a.nsub = nsub;
        a.ms2 = ms2;
        a.S1 = b.S1; a.Bd = b.Bd; a.tw4 = b.tw4x;
        a.nx = p.nx; a.ny = p.ny; a.nz = p.nz; a.Hx = p.Hx; a.ldy = p.ldy; a.ty = ty;
        a.lnl = 0;
        while ((2 << a.lnl) < ty) ++a.lnl;
        launch_x4<T>(p.Px, inv, p.rep[0] > 0, g, x_threads(p, ty), lds4, st, a);
      } else {
        XArgs<T> a;
        a.tbl = tbl; a.ctrl = ctrl; a.stage = stage; a.ms0 = ms0; a.ms1 = ms1; a.nsub = nsub;
        a.ms2 = ms2;
        a.S1 = b.S1; a.Bd = b.Bd; a.tw = b.twx;
        a.nx = p.nx; a.ny = p.ny; a.nz = p.nz; a.Px = p.Px; a.Hx = p.Hx; a.ldy = p.ldy;
        a.ty = ty; a.rad = p.rx;
        const dim3 blk(x_threads(p, ty));
        const size_t ldt = lds + (size_t)p.Px * sizeof(V);   // with the twiddle table
        if (ldt <= kLdsMax) {
          if (inv) hipLaunchKernelGGL((k_fftx_inv<T, false, true>), g, blk, ldt, st, a);
          else hipLaunchKernelGGL((k_fftx_fwd<T, false, true>), g, blk, ldt, st, a);
        } else {
          if (inv) hipLaunchKernelGGL((k_fftx_inv<T, false, false>), g, blk, lds, st, a);
          else hipLaunchKernelGGL((k_fftx_fwd<T, false, false>), g, blk, lds, st, a);
        }
      }
      break;
    }
    case DP_M2: {
      const size_t lds = (size_t)3 * p.nk * p.Py * sizeof(V);
      const dim3 g((p.Hx + p.nk - 1) / p.nk);
      if (p.p2y) {
        M4Args<T> a;
        a.ctrl = ctrl; a.S1 = b.S1; a.K = b.K; a.tw4 = b.tw4y;
        a.ny = p.ny; a.Hx = p.Hx; a.Hy = p.Hy; a.ldy = p.ldy; a.nk = p.nk;
        launch_m4<T>(p.Py, p.rep[1] > 0, g, m2_threads(p), lds, st, a);
      } else {
        M2Args<T> a;
        a.ctrl = ctrl; a.S1 = b.S1; a.K = b.K; a.tw = b.twy;
        a.ny = p.ny; a.Py = p.Py; a.Hx = p.Hx; a.Hy = p.Hy; a.ldy = p.ldy; a.nk = p.nk;
        a.rad = p.ry;
        const size_t ldt = lds + (size_t)p.Py * sizeof(V);
        if (ldt <= kLdsMax)
          hipLaunchKernelGGL((k_ffty_mul2d<T, false, true>), g, dim3(m2_threads(p)), ldt, st, a);
        else
          hipLaunchKernelGGL((k_ffty_mul2d<T, false, false>), g, dim3(m2_threads(p)), lds, st, a);
      }
      break;
    }
    case DP_YF:
    case DP_YI: {
      const bool inv = pass == DP_YI;
      const int nl = inv ? p.nlyi : p.nlyf;
      const int nlines = 3 * p.nz * p.Hx;
      const dim3 g((nlines + nl - 1) / nl);
      const size_t lds = (size_t)nl * p.Py * sizeof(V);
      const cpx<T>* in = inv ? b.S2 : b.S1;
      cpx<T>* out = inv ? b.S1 : b.S2;
      const int nvi = inv ? p.Py : p.ny, ldi = inv ? p.Py : p.ldy;
      const int nvo = inv ? p.ny : p.Py, ldo = inv ? p.ldy : p.Py;
      if (p.p2y) {
        Y4Args<T> a;
        a.ctrl = ctrl; a.in = in; a.out = out; a.tw4 = b.tw4y;
        a.nlines = nlines; a.nvalid_in = nvi; a.ld_in = ldi; a.nvalid_out = nvo; a.ld_out = ldo;
        a.nl = nl;
        launch_y4<T>(p.Py, inv, p.rep[1] > 0, g, y_threads(p, nl), lds, st, a);
      } else {
        YArgs<T> a;
        a.ctrl = ctrl; a.in = in; a.out = out; a.tw = b.twy;
        a.nlines = nlines; a.nvalid_in = nvi; a.ld_in = ldi; a.nvalid_out = nvo; a.ld_out = ldo;
        a.L = p.Py; a.nl = nl; a.rad = p.ry;
        const dim3 blk(y_threads(p, nl));
        const size_t ldt = lds + (size_t)p.Py * sizeof(V);
        if (ldt <= kLdsMax) {
          if (inv) hipLaunchKernelGGL((k_ffty<T, true, false, true>), g, blk, ldt, st, a);
          else hipLaunchKernelGGL((k_ffty<T, false, false, true>), g, blk, ldt, st, a);
        } else {
          if (inv) hipLaunchKernelGGL((k_ffty<T, true, false, false>), g, blk, lds, st, a);
          else hipLaunchKernelGGL((k_ffty<T, false, false, false>), g, blk, lds, st, a);
        }
      }
      break;
    }
    case DP_Z: {
      if (p.p2z) {
        Z4Args<T> a;
        a.ctrl = ctrl; a.S2 = b.S2; a.K = b.K;
        a.nz = p.nz; a.Hx = p.Hx; a.Py = p.Py; a.Hy = p.Hy; a.Hz = p.Hz; a.tk = p.zt;
        const int cpb = p.zt / p.zq;
        const int nblk = ((p.Py + cpb - 1) / cpb) * p.Hx;
        a.nb_pad = round_up(nblk, 8);
        launch_z4<T>(p.Pz, p.zq, p.zw, p.zmode, dim3(a.nb_pad), p.zt, st, a);
      } else {
        ZArgs<T> a;
        a.ctrl = ctrl; a.S2 = b.S2; a.K = b.K; a.tw = b.twz;
        a.nz = p.nz; a.Pz = p.Pz; a.Hx = p.Hx; a.Py = p.Py; a.Hy = p.Hy; a.Hz = p.Hz;
        a.tk = p.tk; a.ls = p.Pz + 1; a.rad = p.rz;
        const dim3 g((p.Py + p.tk - 1) / p.tk, p.Hx), blk(z_threads(p));
        const size_t lds = (size_t)3 * p.tk * (p.Pz + 1) * sizeof(V);
        const size_t ldt = lds + (size_t)p.Pz * sizeof(V);
        if (ldt <= kLdsMax) hipLaunchKernelGGL((k_fftz_mul<T, false, true>), g, blk, ldt, st, a);
        else hipLaunchKernelGGL((k_fftz_mul<T, false, false>), g, blk, lds, st, a);
      }
      break;
    }
  }
}

// ------------------------------------------------------ batched driver --
template <typename T>
struct DemagMulti<T>::Impl {
  // host copies (kept until the next build) and one device allocation
  std::vector<XArgs<T>> xf;
  std::vector<YArgs<T>> yf, yi;
  std::vector<ZArgs<T>> z;
  std::vector<M2Args<T>> m2;
  std::vector<int4> wxf, wxi, wyf, wyi, wz, wm2;
  char* dev = nullptr;
  const XArgs<T>* d_xf = nullptr;
  const XArgs<T>* d_xi = nullptr;
  const YArgs<T>* d_yf = nullptr;
  const YArgs<T>* d_yi = nullptr;
  const ZArgs<T>* d_z = nullptr;
  const M2Args<T>* d_m2 = nullptr;
  const int4 *d_wxf = nullptr, *d_wxi = nullptr, *d_wyf = nullptr, *d_wyi = nullptr,
             *d_wz = nullptr, *d_wm2 = nullptr;
  size_t lds_x = 0, lds_y = 0, lds_z = 0, lds_m2 = 0;
};

template <typename T>
void DemagMulti<T>::release() {
  if (!impl) return;
  if (impl->dev) {
    DeviceLock lk(device_mutex());
    (void)hipFree(impl->dev);
  }
  delete impl;
  impl = nullptr;
}

// largest power of two <= cap (>= 1), at most hi
static int pow2_floor(long cap, int hi) {
  int v = 1;
  while (v < hi && 2L * v <= cap) v *= 2;
  return v;
}

bool demag_multi_fits(const DemagPlan& p) {
  // one line and its twiddle table per block
  const long cap = (long)kMaxE * kMultiThreads;
  if (2L * p.Px > cap || 2L * p.Py > cap) return false;
  if (p.nz == 1) return 4L * p.Py <= cap;
  return 3L * (p.Pz + 1) + p.Pz <= cap;
}

template <typename T>
int DemagMulti<T>::build(const std::vector<DemagMember<T>>& members, hipStream_t st) {
  using V = cpx<T>;
  release();
  if (members.empty()) return 0;
  for (const auto& mb : members)
    if (!demag_multi_fits(*mb.plan)) {
      set_error("batched demag: a pad is too long for one block's lines");
      return MMP_E_ARG;
    }
  impl = new Impl();
  Impl& I = *impl;
  const long cap = (long)kMaxE * kMultiThreads;   // complex elements per block
  for (size_t g = 0; g < members.size(); ++g) {
    const DemagMember<T>& mb = members[g];
    const DemagPlan& p = *mb.plan;
    const int gi = (int)g;
    // x passes: the most rows per block (<= 16) that fit
    // (the twiddle table of the line length sits in LDS beside the lines)
    int ty = 2;
    while (ty < 16 && (long)(ty + 1) * p.Px <= cap && ty < p.ny + (p.ny & 1)) ty *= 2;
    XArgs<T> xa{};
    xa.tbl = mb.tbl; xa.ctrl = mb.ctrl; xa.stage = 0;
    xa.ms0 = mb.ms0; xa.ms1 = mb.ms1; xa.ms2 = mb.ms2; xa.nsub = mb.nsub;
    xa.S1 = mb.bufs.S1; xa.Bd = mb.bufs.Bd; xa.tw = mb.bufs.twx;
    xa.nx = p.nx; xa.ny = p.ny; xa.nz = p.nz; xa.Px = p.Px; xa.Hx = p.Hx; xa.ldy = p.ldy;
    xa.ty = ty; xa.rad = p.rx;
    I.xf.push_back(xa);
    const int xf_idx = (int)I.xf.size() - 1;
    for (int c = 0; c < 3; ++c)
      for (int z = 0; z < p.nz; ++z)
        for (int b = 0; b < (p.ny + ty - 1) / ty; ++b) {
          I.wxf.push_back(make_int4(xf_idx, b, z, c));
          I.wxi.push_back(make_int4(xf_idx, b, z, c));
        }
    I.lds_x = std::max(I.lds_x, (size_t)(ty / 2 + 1) * p.Px * sizeof(V));
    if (p.nz == 1) {
      const int nk = pow2_floor((cap / p.Py - 1) / 3, 64);
      M2Args<T> a{};
      a.ctrl = mb.ctrl; a.S1 = mb.bufs.S1; a.K = mb.bufs.K; a.tw = mb.bufs.twy;
      a.ny = p.ny; a.Py = p.Py; a.Hx = p.Hx; a.Hy = p.Hy; a.ldy = p.ldy; a.nk = nk;
      a.rad = p.ry;
      I.m2.push_back(a);
      const int idx = (int)I.m2.size() - 1;
      for (int b = 0; b < (p.Hx + nk - 1) / nk; ++b) I.wm2.push_back(make_int4(idx, b, 0, 0));
      I.lds_m2 = std::max(I.lds_m2, (size_t)(3 * nk + 1) * p.Py * sizeof(V));
    } else {
      const int nl = pow2_floor(cap / p.Py - 1, 64);
      const int nlines = 3 * p.nz * p.Hx;
      YArgs<T> a{};
      a.ctrl = mb.ctrl; a.tw = mb.bufs.twy; a.nlines = nlines; a.L = p.Py; a.nl = nl;
      a.rad = p.ry;
      YArgs<T> f = a, i = a;
      f.in = mb.bufs.S1; f.out = mb.bufs.S2;
      f.nvalid_in = p.ny; f.ld_in = p.ldy; f.nvalid_out = p.Py; f.ld_out = p.Py;
      i.in = mb.bufs.S2; i.out = mb.bufs.S1;
      i.nvalid_in = p.Py; i.ld_in = p.Py; i.nvalid_out = p.ny; i.ld_out = p.ldy;
      I.yf.push_back(f);
      I.yi.push_back(i);
      const int idx = (int)I.yf.size() - 1;
      for (int b = 0; b < (nlines + nl - 1) / nl; ++b) {
        I.wyf.push_back(make_int4(idx, b, 0, 0));
        I.wyi.push_back(make_int4(idx, b, 0, 0));
      }
      I.lds_y = std::max(I.lds_y, (size_t)(nl + 1) * p.Py * sizeof(V));
      const int tk = pow2_floor((cap - p.Pz) / (3L * (p.Pz + 1)), 64);
      ZArgs<T> za{};
      za.ctrl = mb.ctrl; za.S2 = mb.bufs.S2; za.K = mb.bufs.K; za.tw = mb.bufs.twz;
      za.nz = p.nz; za.Pz = p.Pz; za.Hx = p.Hx; za.Py = p.Py; za.Hy = p.Hy; za.Hz = p.Hz;
      za.tk = tk; za.ls = p.Pz + 1; za.rad = p.rz;
      I.z.push_back(za);
      const int zi = (int)I.z.size() - 1;
      for (int kx = 0; kx < p.Hx; ++kx)
        for (int b = 0; b < (p.Py + tk - 1) / tk; ++b) I.wz.push_back(make_int4(zi, b, kx, 0));
      I.lds_z = std::max(I.lds_z, ((size_t)3 * tk * (p.Pz + 1) + p.Pz) * sizeof(V));
    }
  }
  // one device allocation, 256-byte aligned segments
  size_t off = 0;
  auto seg = [&](size_t bytes) {
    const size_t o = off;
    off += (bytes + 255) / 256 * 256;
    return o;
  };
  const size_t o_xf = seg(I.xf.size() * sizeof(XArgs<T>));
  const size_t o_yf = seg(I.yf.size() * sizeof(YArgs<T>));
  const size_t o_yi = seg(I.yi.size() * sizeof(YArgs<T>));
  const size_t o_z = seg(I.z.size() * sizeof(ZArgs<T>));
  const size_t o_m2 = seg(I.m2.size() * sizeof(M2Args<T>));
  const size_t o_wxf = seg(I.wxf.size() * sizeof(int4));
  const size_t o_wxi = seg(I.wxi.size() * sizeof(int4));
  const size_t o_wyf = seg(I.wyf.size() * sizeof(int4));
  const size_t o_wyi = seg(I.wyi.size() * sizeof(int4));
  const size_t o_wz = seg(I.wz.size() * sizeof(int4));
  const size_t o_wm2 = seg(I.wm2.size() * sizeof(int4));
  hipError_t ae;
  {
    DeviceLock lk(device_mutex());
    ae = hipMalloc(&I.dev, off);
  }
  if (ae != hipSuccess) {
    I.dev = nullptr;
    release();
    set_error("device allocation failed (batched demag tables)");
    return MMP_E_NOMEM;
  }
  auto put = [&](size_t o, const void* src, size_t bytes) {
    return bytes ? hipMemcpyAsync(I.dev + o, src, bytes, hipMemcpyHostToDevice, st) : hipSuccess;
  };
  hipError_t e = hipSuccess;
  for (auto r : {put(o_xf, I.xf.data(), I.xf.size() * sizeof(XArgs<T>)),
                 put(o_yf, I.yf.data(), I.yf.size() * sizeof(YArgs<T>)),
                 put(o_yi, I.yi.data(), I.yi.size() * sizeof(YArgs<T>)),
                 put(o_z, I.z.data(), I.z.size() * sizeof(ZArgs<T>)),
                 put(o_m2, I.m2.data(), I.m2.size() * sizeof(M2Args<T>)),
                 put(o_wxf, I.wxf.data(), I.wxf.size() * sizeof(int4)),
                 put(o_wxi, I.wxi.data(), I.wxi.size() * sizeof(int4)),
                 put(o_wyf, I.wyf.data(), I.wyf.size() * sizeof(int4)),
                 put(o_wyi, I.wyi.data(), I.wyi.size() * sizeof(int4)),
                 put(o_wz, I.wz.data(), I.wz.size() * sizeof(int4)),
                 put(o_wm2, I.wm2.data(), I.wm2.size() * sizeof(int4))})
    if (r != hipSuccess) e = r;
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    release();
    set_error(std::string("batched demag tables: ") + hipGetErrorString(e));
    return MMP_E_HIP;
  }
  // the x inverse pass reads the same arguments as the forward one
  I.d_xf = reinterpret_cast<const XArgs<T>*>(I.dev + o_xf);
  I.d_xi = I.d_xf;
  I.d_yf = reinterpret_cast<const YArgs<T>*>(I.dev + o_yf);
  I.d_yi = reinterpret_cast<const YArgs<T>*>(I.dev + o_yi);
  I.d_z = reinterpret_cast<const ZArgs<T>*>(I.dev + o_z);
  I.d_m2 = reinterpret_cast<const M2Args<T>*>(I.dev + o_m2);
  I.d_wxf = reinterpret_cast<const int4*>(I.dev + o_wxf);
  I.d_wxi = reinterpret_cast<const int4*>(I.dev + o_wxi);
  I.d_wyf = reinterpret_cast<const int4*>(I.dev + o_wyf);
  I.d_wyi = reinterpret_cast<const int4*>(I.dev + o_wyi);
  I.d_wz = reinterpret_cast<const int4*>(I.dev + o_wz);
  I.d_wm2 = reinterpret_cast<const int4*>(I.dev + o_wm2);
  return 0;
}

template <typename T>
void DemagMulti<T>::launch(int stage, hipStream_t st) const {
  if (!impl) return;
  const Impl& I = *impl;
  const dim3 b(kMultiThreads);
  hipLaunchKernelGGL((k_fftx_fwd_multi<T>), dim3((unsigned)I.wxf.size()), b, I.lds_x, st, I.d_xf,
                     I.d_wxf, stage);
  if (!I.wm2.empty())
    hipLaunchKernelGGL((k_ffty_mul2d_multi<T>), dim3((unsigned)I.wm2.size()), b, I.lds_m2, st,
                       I.d_m2, I.d_wm2);
  if (!I.wyf.empty()) {
    hipLaunchKernelGGL((k_ffty_multi<T, false>), dim3((unsigned)I.wyf.size()), b, I.lds_y, st,
                       I.d_yf, I.d_wyf);
    hipLaunchKernelGGL((k_fftz_mul_multi<T>), dim3((unsigned)I.wz.size()), b, I.lds_z, st, I.d_z,
                       I.d_wz);
    hipLaunchKernelGGL((k_ffty_multi<T, true>), dim3((unsigned)I.wyi.size()), b, I.lds_y, st,
                       I.d_yi, I.d_wyi);
  }
  hipLaunchKernelGGL((k_fftx_inv_multi<T>), dim3((unsigned)I.wxi.size()), b, I.lds_x, st, I.d_xi,
                     I.d_wxi);
}

template class DemagMulti<float>;
template class DemagMulti<double>;

static const int kPassProf[DP_COUNT] = {P_FFTX_FWD, P_FFTY_FWD, P_FFTZ_MUL,
                                        P_FFTY_INV, P_FFTX_INV, P_FFTY_MUL2D};

static int demag_passes(const DemagPlan& p, int* out) {
  int n = 0;
  out[n++] = DP_XF;
  if (p.nz == 1) {
    out[n++] = DP_M2;
  } else {
    out[n++] = DP_YF;
    out[n++] = DP_Z;
    out[n++] = DP_YI;
  }
  out[n++] = DP_XI;
  return n;
}

// --------------------------------------------------------------- driver --
template <typename T>
void demag_field(const DemagPlan& p, const DemagBufs<T>& b, const Table<T>* tbl, int stage,
                 const Ctrl* ctrl, T ms0, T ms1, int nsub, hipStream_t st, Prof* prof, T ms2) {
  int passes[DP_COUNT];
  const int n = demag_passes(p, passes);
  for (int i = 0; i < n; ++i) {
    ProfScope ps(prof, kPassProf[passes[i]], st);
    demag_pass<T>(passes[i], p, b, tbl, stage, ctrl, ms0, ms1, nsub, st, ms2);
  }
}

// ------------------------------------------------------------ autotuner --
// Mean time of `reps` launches of the passes in seq[0..ns) after one warm-up
// launch of the last; negative when a launch fails. The tuner times each
// candidate of a pass right after the pass before it in an evaluation (the
// first pass after the last one), so the candidate meets the caches as it
// does there (the pair's time ranks the candidates as their own would).
template <typename T>
static double time_passes(const int* seq, int ns, const DemagPlan& p, const DemagBufs<T>& b,
                          const Table<T>* tbl, T ms0, T ms1, int nsub, hipStream_t st, int reps,
                          T ms2) {
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return -1.0;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return -1.0;
  }
  double ms = -1.0;
  demag_pass<T>(seq[ns - 1], p, b, tbl, 1, nullptr, ms0, ms1, nsub, st, ms2);
  if (hipGetLastError() == hipSuccess && hipEventRecord(e0, st) == hipSuccess) {
    for (int r = 0; r < reps; ++r)
      for (int j = 0; j < ns; ++j) demag_pass<T>(seq[j], p, b, tbl, 1, nullptr, ms0, ms1, nsub, st, ms2);
    float f = 0.f;
    if (hipGetLastError() == hipSuccess && hipEventRecord(e1, st) == hipSuccess &&
        hipEventSynchronize(e1) == hipSuccess && hipEventElapsedTime(&f, e0, e1) == hipSuccess)
      ms = (double)f / reps;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return ms;
}

template <typename T>
double demag_tune(DemagPlan* pp, const DemagBufs<T>& b, const Table<T>* tbl, T ms0, T ms1,
                  int nsub, hipStream_t st, T ms2) {
  constexpr int rb = (int)sizeof(T);
  DemagPlan best = *pp;
  int passes[DP_COUNT];
  const int n = demag_passes(best, passes);
  // launches per timing: enough to average out launch jitter on small grids
  // and run-to-run spread of a few percent on large ones
  const long work = (long)best.Hx * best.Py * best.Pz;
  const int reps = work >= (1L << 22) ? 8 : work >= (1L << 16) ? 10 : 30;
  for (int i = 0; i < n; ++i) {
    const int pass = passes[i];
    std::vector<DemagPlan> cand;
    auto add = [&](DemagPlan c) {
      if (demag_plan_check(c, rb) == 0) cand.push_back(c);
    };
    switch (pass) {
      case DP_XF:
      case DP_XI:
        for (int ty = 2; ty <= 16; ty *= 2) {
          DemagPlan c = best;
          (pass == DP_XF ? c.tyf : c.tyi) = ty;
          add(c);
        }
        break;
      case DP_YF:
      case DP_YI:
        for (int nl = 1; nl <= 64; nl *= 2) {
          DemagPlan c = best;
          (pass == DP_YF ? c.nlyf : c.nlyi) = nl;
          add(c);
        }
        break;
      case DP_M2:
        for (int k = 1; k <= 64; k *= 2) {
          DemagPlan c = best;
          c.nk = k;
          add(c);
        }
        break;
      case DP_Z:
        if (best.p2z) {
          for (int q = 1; q <= 4; q *= 2)
            for (int w = 1; w <= 4; w *= 2)
              for (int t = 64; t <= 256; t *= 2)
                for (int k = 0; k <= 1; ++k) {
                  DemagPlan c = best;
                  c.zq = q; c.zw = w; c.zt = t; c.zmode = k;
                  add(c);
                }
        } else {
          for (int tk = 1; tk <= 64; tk *= 2) {
            DemagPlan c = best;
            c.tk = tk;
            add(c);
          }
        }
        break;
    }
    double bt = -1.0;
    for (const DemagPlan& c : cand) {
      // the first pass follows the last one of the previous evaluation
      const int pair[2] = {passes[i > 0 ? i - 1 : n - 1], pass};
      const double t = time_passes<T>(pair, n > 1 ? 2 : 1, c, b, tbl, ms0, ms1, nsub, st, reps,
                                      ms2);
      if (t < 0.0) continue;
      if (bt < 0.0 || t < bt) {
        bt = t;
        best = c;
      }
    }
    if (bt < 0.0) return -1.0;
  }
  // the reported estimate: one whole evaluation with the chosen plan
  const double total = time_passes<T>(passes, n, best, b, tbl, ms0, ms1, nsub, st, reps, ms2);
  if (total < 0.0) return -1.0;
  *pp = best;
  return total;
}

#define INST(T)                                                                                 \
  template void demag_field<T>(const DemagPlan&, const DemagBufs<T>&, const Table<T>*, int,      \
                               const Ctrl*, T, T, int, hipStream_t, Prof*, T);                  \
  template void demag_pass<T>(int, const DemagPlan&, const DemagBufs<T>&, const Table<T>*, int,  \
                              const Ctrl*, T, T, int, hipStream_t, T);                          \
  template double demag_tune<T>(DemagPlan*, const DemagBufs<T>&, const Table<T>*, T, T, int,    \
                                hipStream_t, T);
INST(float)
INST(double)
#undef INST

}  // namespace mmp
