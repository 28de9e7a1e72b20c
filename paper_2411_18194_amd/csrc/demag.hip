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
  T ms0, ms1;
  int nsub;
  cpx<T>* S1;
  T* Bd;
  const cpx<T>* tw;
  int nx, ny, nz, Px, Hx, ldy, ty;
  Rad rad;
};

template <typename T, bool P2>
__global__ void k_fftx_fwd(XArgs<T> a) {
  using V = cpx<T>;
  if (ctrl_stopped(a.ctrl)) return;
  extern __shared__ char smem_raw[];
  V* buf = reinterpret_cast<V*>(smem_raw);
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int c = blockIdx.z, z = blockIdx.y, y0 = blockIdx.x * a.ty;
  const int nl = a.ty >> 1;
  const long N = (long)a.nx * a.ny * a.nz;
  const T* m = stage_in(a.tbl, a.stage);
  const T* m0 = m + (long)c * N + (long)z * a.ny * a.nx;
  const T* m1 = m0 + 3 * N;
  for (int idx = tid; idx < nl * a.Px; idx += nthr) {
    const int q = idx / a.Px, x = idx - q * a.Px;
    const int ya = y0 + 2 * q, yb = ya + 1;
    T re = 0, im = 0;
    if (x < a.nx) {
      if (ya < a.ny) {
        re = a.ms0 * m0[(long)ya * a.nx + x];
        if (a.nsub == 2) re += a.ms1 * m1[(long)ya * a.nx + x];
      }
      if (yb < a.ny) {
        im = a.ms0 * m0[(long)yb * a.nx + x];
        if (a.nsub == 2) im += a.ms1 * m1[(long)yb * a.nx + x];
      }
    }
    buf[q * a.Px + x] = cmk<T>(re, im);
  }
  __syncthreads();
  lds_fft<T, false, P2>(buf, a.tw, a.Px, nl, a.Px, a.rad.n, a.rad.code, tid, nthr);
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

template <typename T, bool P2>
__global__ void k_fftx_inv(XArgs<T> a) {
  using V = cpx<T>;
  if (ctrl_stopped(a.ctrl)) return;
  extern __shared__ char smem_raw[];
  V* buf = reinterpret_cast<V*>(smem_raw);
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int c = blockIdx.z, z = blockIdx.y, y0 = blockIdx.x * a.ty;
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
  __syncthreads();
  lds_fft<T, true, P2>(buf, a.tw, a.Px, nl, a.Px, a.rad.n, a.rad.code, tid, nthr);
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

template <typename T, bool INV, bool P2>
__global__ void k_ffty(YArgs<T> a) {
  using V = cpx<T>;
  if (ctrl_stopped(a.ctrl)) return;
  extern __shared__ char smem_raw[];
  V* buf = reinterpret_cast<V*>(smem_raw);
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int l0 = blockIdx.x * a.nl;
  for (int idx = tid; idx < a.nl * a.L; idx += nthr) {
    const int q = idx / a.L, e = idx - q * a.L;
    const int gl = l0 + q;
    V v = cmk<T>(0, 0);
    if (gl < a.nlines && e < a.nvalid_in) v = a.in[(long)gl * a.ld_in + e];
    buf[q * a.L + e] = v;
  }
  __syncthreads();
  lds_fft<T, INV, P2>(buf, a.tw, a.L, a.nl, a.L, a.rad.n, a.rad.code, tid, nthr);
  for (int idx = tid; idx < a.nl * a.nvalid_out; idx += nthr) {
    const int q = idx / a.nvalid_out, e = idx - q * a.nvalid_out;
    const int gl = l0 + q;
    if (gl < a.nlines) a.out[(long)gl * a.ld_out + e] = buf[q * a.L + e];
  }
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

template <typename T, bool P2>
__global__ void k_ffty_mul2d(M2Args<T> a) {
  using V = cpx<T>;
  if (ctrl_stopped(a.ctrl)) return;
  extern __shared__ char smem_raw[];
  V* buf = reinterpret_cast<V*>(smem_raw);
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int kx0 = blockIdx.x * a.nk;
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
  __syncthreads();
  lds_fft<T, false, P2>(buf, a.tw, L, nl, L, a.rad.n, a.rad.code, tid, nthr);
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
  lds_fft<T, true, P2>(buf, a.tw, L, nl, L, a.rad.n, a.rad.code, tid, nthr);
  for (int idx = tid; idx < nl * a.ny; idx += nthr) {
    const int line = idx / a.ny, e = idx - line * a.ny;
    const int c = line / a.nk, j = line - c * a.nk;
    const int kx = kx0 + j;
    if (kx < a.Hx) a.S1[((long)c * a.Hx + kx) * a.ldy + e] = buf[line * L + e];
  }
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

template <typename T, bool P2>
__global__ void k_fftz_mul(ZArgs<T> a) {
  using V = cpx<T>;
  if (ctrl_stopped(a.ctrl)) return;
  extern __shared__ char smem_raw[];
  V* buf = reinterpret_cast<V*>(smem_raw);
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int kx = blockIdx.y, ky0 = blockIdx.x * a.tk;
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
  __syncthreads();
  lds_fft<T, false, P2>(buf, a.tw, L, nl, a.ls, a.rad.n, a.rad.code, tid, nthr);
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
  lds_fft<T, true, P2>(buf, a.tw, L, nl, a.ls, a.rad.n, a.rad.code, tid, nthr);
  V* obase = a.S2 + (long)kx * a.Py + ky0;
  for (int idx = tid; idx < 3 * a.tk * a.nz; idx += nthr) {
    const int j = idx % a.tk;
    const int r = idx / a.tk;
    const int z = r % a.nz, c = r / a.nz;
    if (ky0 + j < a.Py) obase[c * cstride + z * zstride + j] = buf[(c * a.tk + j) * a.ls + z];
  }
}

// ------------------------------------------------------------------ plan --
static int threads_for(long elems) {
  long t = (elems + kMaxE - 1) / kMaxE;
  t = (t + 63) / 64 * 64;
  if (t < 64) t = 64;
  return (int)t;
}

int demag_plan(int nx, int ny, int nz, int real_bytes, DemagPlan* p) {
  DemagPlan d;
  d.nx = nx; d.ny = ny; d.nz = nz;
  d.Px = smooth_pad(nx); d.Py = smooth_pad(ny); d.Pz = smooth_pad(nz);
  if (d.Px > 4096 || d.Py > 4096 || d.Pz > 4096) return -1;
  d.Hx = d.Px / 2 + 1; d.Hy = d.Py / 2 + 1; d.Hz = d.Pz / 2 + 1;
  int rr[3][16];
  const int nrx = fft_radices(d.Px, rr[0]);
  const int nry = fft_radices(d.Py, rr[1]);
  const int nrz = fft_radices(d.Pz, rr[2]);
  if (nrx < 0 || nry < 0 || nrz < 0 || nrx > 15 || nry > 15 || nrz > 15) return -1;
  d.rx = make_rad(rr[0], nrx);
  d.ry = make_rad(rr[1], nry);
  d.rz = make_rad(rr[2], nrz);
  // complex elements one block may hold in LDS (64 KiB)
  const long cap = 65536 / (2 * real_bytes);
  // x passes: ty rows (pairs) per block
  int ty = 2;
  while (ty < 16 && (long)(ty) * d.Px <= cap && ty < ny + (ny & 1)) ty *= 2;
  if ((long)(ty / 2) * d.Px > cap) ty /= 2;
  if (ty < 2) ty = 2;
  d.ty = ty;
  d.thr_x = threads_for((long)(ty / 2) * d.Px);
  d.ldy = round_up(ny, ty);
  // y passes: lines per block
  int nl = 1;
  while (nl < 8 && (long)(2 * nl) * d.Py <= cap && (long)(2 * nl) * d.Py <= 4096) nl *= 2;
  d.nly = nl;
  d.thr_y = threads_for((long)nl * d.Py);
  // 2-D fused pass: kx columns per block
  int nk = 1;
  while (nk < 64 && (long)3 * (2 * nk) * d.Py <= cap && (long)3 * (2 * nk) * d.Py <= 6144) nk *= 2;
  d.nk2 = nk;
  d.thr_m2 = threads_for((long)3 * nk * d.Py);
  // z pass: ky per block, padded line stride against bank conflicts
  d.lsz = d.Pz + 1;
  int tk = 64;
  while (tk > 1 && (long)3 * tk * d.lsz > cap) tk /= 2;
  d.tk = tk;
  d.thr_z = threads_for((long)3 * tk * d.Pz);
  if (d.thr_x > 1024 || d.thr_y > 1024 || d.thr_m2 > 1024 || d.thr_z > 1024) return -1;
  // power-of-two axes: register four-step kernels (FP64 only up to 2048
  // points per line, the z column up to 32 points)
  const int lmax = real_bytes == 8 ? 2048 : 4096;
  d.p2x = is_pow2(d.Px) && d.Px <= lmax;
  d.p2y = is_pow2(d.Py) && d.Py <= lmax;
  // the register z pass holds three columns per thread: up to 32 points in
  // FP32, 16 in FP64
  d.p2z = is_pow2(d.Pz) && d.Pz <= (real_bytes == 8 ? 16 : 32);
  {
    const int l2 = split_l2(d.Py);
    int n = 1;
    while (n < 64 && (long)(2 * n) * d.Py <= cap && 2 * n * l2 <= 256) n *= 2;
    d.nly4 = n;
    int k = 1;
    while (k < 64 && (long)3 * (2 * k) * d.Py <= cap && 3 * (2 * k) * l2 <= 256) k *= 2;
    d.nk4 = k;
    // z pass: threads (ky columns) per block
    d.tk4 = real_bytes == 8 ? 64 : 128;
    // the x rows per block also bound the four-step block to 256 threads
    if (d.p2x)
      while ((d.ty / 2) * split_l2(d.Px) > 256) d.ty /= 2;
    d.ldy = round_up(ny, d.ty);
    if (3 * d.nk4 * l2 > 256 || d.nly4 * l2 > 256 || d.tk4 > 256) return -1;
  }
  d.s1_elems = (size_t)3 * nz * d.Hx * d.ldy;
  d.s2_elems = nz > 1 ? (size_t)3 * nz * d.Hx * d.Py : 0;
  d.k_elems = (size_t)6 * d.Hz * d.Hx * d.Hy;
  *p = d;
  return 0;
}

// --------------------------------------------------------------- driver --
template <typename T>
void demag_field(const DemagPlan& p, const DemagBufs<T>& b, const Table<T>* tbl, int stage,
                 const Ctrl* ctrl, T ms0, T ms1, int nsub, hipStream_t st, Prof* prof) {
  using V = cpx<T>;
  const dim3 gx((p.ny + p.ty - 1) / p.ty, p.nz, 3);
  const size_t lds_x = (size_t)(p.ty / 2) * p.Px * sizeof(V);
  XArgs<T> xa;
  xa.tbl = tbl; xa.ctrl = ctrl; xa.stage = stage; xa.ms0 = ms0; xa.ms1 = ms1; xa.nsub = nsub;
  xa.S1 = b.S1; xa.Bd = b.Bd; xa.tw = b.twx;
  xa.nx = p.nx; xa.ny = p.ny; xa.nz = p.nz; xa.Px = p.Px; xa.Hx = p.Hx; xa.ldy = p.ldy;
  xa.ty = p.ty; xa.rad = p.rx;
  X4Args<T> x4;
  x4.tbl = tbl; x4.ctrl = ctrl; x4.stage = stage; x4.ms0 = ms0; x4.ms1 = ms1; x4.nsub = nsub;
  x4.S1 = b.S1; x4.Bd = b.Bd; x4.tw4 = b.tw4x;
  x4.nx = p.nx; x4.ny = p.ny; x4.nz = p.nz; x4.Hx = p.Hx; x4.ldy = p.ldy; x4.ty = p.ty;
  const int thr_x4 = (p.ty / 2) * split_l2(p.Px);
  {
    ProfScope ps(prof, P_FFTX_FWD, st);
    if (p.p2x) launch_x4<T>(p.Px, false, gx, thr_x4, lds_x, st, x4);
    else hipLaunchKernelGGL((k_fftx_fwd<T, false>), gx, dim3(p.thr_x), lds_x, st, xa);
  }
  if (p.nz == 1) {
    ProfScope ps(prof, P_FFTY_MUL2D, st);
    if (p.p2y) {
      M4Args<T> m4;
      m4.ctrl = ctrl; m4.S1 = b.S1; m4.K = b.K; m4.tw4 = b.tw4y;
      m4.ny = p.ny; m4.Hx = p.Hx; m4.Hy = p.Hy; m4.ldy = p.ldy; m4.nk = p.nk4;
      launch_m4<T>(p.Py, dim3((p.Hx + p.nk4 - 1) / p.nk4), 3 * p.nk4 * split_l2(p.Py),
                   (size_t)3 * p.nk4 * p.Py * sizeof(V), st, m4);
    } else {
      M2Args<T> ma;
      ma.ctrl = ctrl; ma.S1 = b.S1; ma.K = b.K; ma.tw = b.twy;
      ma.ny = p.ny; ma.Py = p.Py; ma.Hx = p.Hx; ma.Hy = p.Hy; ma.ldy = p.ldy; ma.nk = p.nk2;
      ma.rad = p.ry;
      hipLaunchKernelGGL((k_ffty_mul2d<T, false>), dim3((p.Hx + p.nk2 - 1) / p.nk2),
                         dim3(p.thr_m2), (size_t)3 * p.nk2 * p.Py * sizeof(V), st, ma);
    }
  } else {
    const int nlines = 3 * p.nz * p.Hx;
    YArgs<T> ya;
    ya.ctrl = ctrl; ya.in = b.S1; ya.out = b.S2; ya.tw = b.twy;
    ya.nlines = nlines; ya.nvalid_in = p.ny; ya.ld_in = p.ldy; ya.nvalid_out = p.Py;
    ya.ld_out = p.Py; ya.L = p.Py; ya.nl = p.nly; ya.rad = p.ry;
    const dim3 gy((nlines + p.nly - 1) / p.nly);
    const size_t lds_y = (size_t)p.nly * p.Py * sizeof(V);
    Y4Args<T> y4;
    y4.ctrl = ctrl; y4.in = b.S1; y4.out = b.S2; y4.tw4 = b.tw4y;
    y4.nlines = nlines; y4.nvalid_in = p.ny; y4.ld_in = p.ldy; y4.nvalid_out = p.Py;
    y4.ld_out = p.Py; y4.nl = p.nly4;
    const dim3 gy4((nlines + p.nly4 - 1) / p.nly4);
    const int thr_y4 = p.nly4 * split_l2(p.Py);
    const size_t lds_y4 = (size_t)p.nly4 * p.Py * sizeof(V);
    {
      ProfScope ps(prof, P_FFTY_FWD, st);
      if (p.p2y) launch_y4<T>(p.Py, false, gy4, thr_y4, lds_y4, st, y4);
      else hipLaunchKernelGGL((k_ffty<T, false, false>), gy, dim3(p.thr_y), lds_y, st, ya);
    }
    {
      ProfScope ps(prof, P_FFTZ_MUL, st);
      if (p.p2z) {
        Z4Args<T> z4;
        z4.ctrl = ctrl; z4.S2 = b.S2; z4.K = b.K;
        z4.nz = p.nz; z4.Hx = p.Hx; z4.Py = p.Py; z4.Hy = p.Hy; z4.Hz = p.Hz; z4.tk = p.tk4;
        const int zthr = p.tk4;
        const int nblk = ((p.Py + zthr - 1) / zthr) * p.Hx;
        z4.nb_pad = round_up(nblk, 8);
        launch_z4<T>(p.Pz, dim3(z4.nb_pad), zthr, 0, st, z4);
      } else {
        ZArgs<T> za;
        za.ctrl = ctrl; za.S2 = b.S2; za.K = b.K; za.tw = b.twz;
        za.nz = p.nz; za.Pz = p.Pz; za.Hx = p.Hx; za.Py = p.Py; za.Hy = p.Hy; za.Hz = p.Hz;
        za.tk = p.tk; za.ls = p.lsz; za.rad = p.rz;
        hipLaunchKernelGGL((k_fftz_mul<T, false>), dim3((p.Py + p.tk - 1) / p.tk, p.Hx),
                           dim3(p.thr_z), (size_t)3 * p.tk * p.lsz * sizeof(V), st, za);
      }
    }
    {
      ProfScope ps(prof, P_FFTY_INV, st);
      if (p.p2y) {
        Y4Args<T> yi = y4;
        yi.in = b.S2; yi.out = b.S1; yi.nvalid_in = p.Py; yi.ld_in = p.Py;
        yi.nvalid_out = p.ny; yi.ld_out = p.ldy;
        launch_y4<T>(p.Py, true, gy4, thr_y4, lds_y4, st, yi);
      } else {
        YArgs<T> yi = ya;
        yi.in = b.S2; yi.out = b.S1; yi.nvalid_in = p.Py; yi.ld_in = p.Py;
        yi.nvalid_out = p.ny; yi.ld_out = p.ldy;
        hipLaunchKernelGGL((k_ffty<T, true, false>), gy, dim3(p.thr_y), lds_y, st, yi);
      }
    }
  }
  {
    ProfScope ps(prof, P_FFTX_INV, st);
    if (p.p2x) launch_x4<T>(p.Px, true, gx, thr_x4, lds_x, st, x4);
    else hipLaunchKernelGGL((k_fftx_inv<T, false>), gx, dim3(p.thr_x), lds_x, st, xa);
  }
}

template void demag_field<float>(const DemagPlan&, const DemagBufs<float>&, const Table<float>*,
                                 int, const Ctrl*, float, float, int, hipStream_t, Prof*);
template void demag_field<double>(const DemagPlan&, const DemagBufs<double>&,
                                  const Table<double>*, int, const Ctrl*, double, double, int,
                                  hipStream_t, Prof*);

}  // namespace mmp
