// Power-of-two demag passes built on register FFTs (see fft4.h).
//
// Same pass structure and memory layout as the mixed-radix passes in
// demag.hip; only the in-block transform differs: each line is a four-step
// transform (two register FFTs and one swizzled LDS transpose) and the z
// pass holds a whole column per thread.  Loads and stores of lines are
// coalesced across the L2 threads of a line.
#include "demag4.h"
#include "fft4.h"

#include <type_traits>

namespace mmp {

template <typename T>
__global__ void k_twiddles4(cpx<T>* tw, int L1, int L2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= L1 * L2) return;
  const int k1 = i / L2, t = i - k1 * L2;
  double s, c;
  sincospi(-2.0 * (double)(t * k1) / (double)(L1 * L2), &s, &c);
  tw[i] = cmk<T>((T)c, (T)s);
}

int split_l2(int L) {
  int lg = 0;
  while ((1 << lg) < L) ++lg;
  return 1 << (lg / 2);
}

template <typename T>
void build_twiddles4(cpx<T>* tw, int L, hipStream_t st) {
  const int L2 = split_l2(L), L1 = L / L2;
  hipLaunchKernelGGL(k_twiddles4<T>, dim3((L + 255) / 256), dim3(256), 0, st, tw, L1, L2);
}
template void build_twiddles4<float>(cpx<float>*, int, hipStream_t);
template void build_twiddles4<double>(cpx<double>*, int, hipStream_t);

// step 1: L1-point register FFT, inter-step twiddle, swizzled LDS row store.
// HZ: the line is zero-padded to at least twice its data (every pow-2 pad
// P >= 2n - 1 is even, so P >= 2n), so v[L1/2 ..) is zero and not read.
template <typename T, int L1, int L2, bool INV, bool HZ = false>
__device__ __forceinline__ void fs_step1(cpx<T>* v, cpx<T>* line, const cpx<T>* __restrict__ tw4,
                                         int t) {
  if constexpr (HZ && L1 >= 2) reg_fft_hz<T, L1, INV>(v);
  else reg_fft<T, L1, INV>(v);
#pragma unroll
  for (int k1 = 0; k1 < L1; ++k1) {
    cpx<T> x = v[bitrev<L1>(k1)];
    if (k1 > 0) {
      cpx<T> w = tw4[k1 * L2 + t];
      if (INV) w.y = -w.y;
      x = cmul(x, w);
    }
    line[k1 * L2 + (t ^ (k1 & (L2 - 1)))] = x;
  }
}

// step 3: L2-point register FFTs of the swizzled columns owned by thread t;
// u[i][bitrev<L2>(k2)] = X[t + L2 i + L1 k2]
template <typename T, int L1, int L2, bool INV>
__device__ __forceinline__ void fs_step3(cpx<T> (*u)[L2], const cpx<T>* line, int t) {
#pragma unroll
  for (int i = 0; i < L1 / L2; ++i) {
    const int k1 = t + L2 * i;
#pragma unroll
    for (int n2 = 0; n2 < L2; ++n2) u[i][n2] = line[k1 * L2 + (n2 ^ (k1 & (L2 - 1)))];
    reg_fft<T, L2, INV>(u[i]);
  }
}

// two consecutive complex values as one 16-byte access where they fit (the
// load is the x inverse pass's single read of its spectrum: non-temporal)
template <typename T>
__device__ __forceinline__ void store2(cpx<T>* o, cpx<T> a, cpx<T> b) {
  if constexpr (sizeof(cpx<T>) == 8) {
    float4 v;
    v.x = a.x; v.y = a.y; v.z = b.x; v.w = b.y;
    *reinterpret_cast<float4*>(o) = v;
  } else {
    o[0] = a;
    o[1] = b;
  }
}
template <typename T>
__device__ __forceinline__ void load2(const cpx<T>* i, cpx<T>& a, cpx<T>& b) {
  if constexpr (sizeof(cpx<T>) == 8) {
    const nt_f4 v = __builtin_nontemporal_load(reinterpret_cast<const nt_f4*>(i));
    a = cmk<T>(v.x, v.y);
    b = cmk<T>(v.z, v.w);
  } else {
    a = ntload(i);
    b = ntload(i + 1);
  }
}

// ------------------------------------------------------------ y lines --
// FULL: the input line fills the whole transform length (a periodic axis);
// otherwise a forward line is zero-padded to at least twice its data.
template <typename T, int L1, int L2, bool INV, bool FULL>
__global__ __launch_bounds__(256) void k4_ffty(Y4Args<T> a) {
  using V = cpx<T>;
  if (ctrl_stopped(a.ctrl)) return;
  constexpr int L = L1 * L2;
  extern __shared__ char smem_raw[];
  V* lds = reinterpret_cast<V*>(smem_raw);
  const int t = threadIdx.x % L2, q = threadIdx.x / L2;
  const int gl = blockIdx.x * a.nl + q;
  const bool valid = gl < a.nlines;
  V* line = lds + q * L;
  // loads are unconditional (clamped to element 0 of line 0) and zeroed
  // afterwards, so they all go out before the first wait
  const V* in = a.in + (long)(valid ? gl : 0) * a.ld_in;
  V v[L1];
  constexpr bool HZ = !INV && !FULL;
  constexpr int NLOAD = (HZ && L1 >= 2) ? L1 / 2 : L1;
#pragma unroll
  for (int n1 = 0; n1 < NLOAD; ++n1) {
    const int idx = L2 * n1 + t;
    v[n1] = ntload(in + (idx < a.nvalid_in ? idx : 0));
  }
#pragma unroll
  for (int n1 = 0; n1 < NLOAD; ++n1)
    if (!valid || L2 * n1 + t >= a.nvalid_in) v[n1] = cmk<T>(0, 0);
  fs_step1<T, L1, L2, INV, HZ>(v, line, a.tw4, t);
  __syncthreads();
  V u[L1 / L2][L2];
  fs_step3<T, L1, L2, INV>(u, line, t);
  if (valid) {
    V* out = a.out + (long)gl * a.ld_out;
#pragma unroll
    for (int i = 0; i < L1 / L2; ++i)
#pragma unroll
      for (int k2 = 0; k2 < L2; ++k2) {
        const int k = t + L2 * i + L1 * k2;
        if (k < a.nvalid_out) {
          // the forward spectrum is read once, by the z pass
          if (INV) out[k] = u[i][bitrev<L2>(k2)];
          else ntstore(out + k, u[i][bitrev<L2>(k2)]);
        }
      }
  }
}

// ------------------------------------------------------------- x rows --
// The x passes pack and unpack the two real rows of a line in natural order
// with one (line, kx) per thread, eight lines of a block side by side: lines
// 8 KiB apart put element kx of every line in the same LDS bank.  Element e
// of line q therefore sits at e ^ xsw<L>(q): a permutation within aligned
// groups of 32 (so runs of 32 consecutive elements stay conflict-free) that
// spreads the lines over the banks (lines shorter than 32 keep their order).
template <int L>
__device__ __forceinline__ int xsw(int q) { return L >= 32 ? (q & 3) << 3 : 0; }

// Makes the N complex values in registers at this point of the program: the
// compiler can neither sink their computation below it nor hoist later uses
// above it (an empty asm that reads and rewrites each register).  Between
// the phases of a register z pass this keeps the forward transforms, the
// kernel products and the inverse transforms from interleaving, which would
// hold more values live at once than the 256 registers of two waves per SIMD.
template <int N, typename T>
__device__ __forceinline__ void pin_regs(cpx<T>* v) {
#pragma unroll
  for (int i = 0; i < N; ++i) asm volatile("" : "+v"(v[i].x), "+v"(v[i].y));
}

// The half-LDS x forward pass after the loads: register FFTs and twiddles
// of step 1, the transpose in two halves of rows, the step-3 FFTs, then the
// unpack of the two real spectra in two halves of the spectrum.
template <int L>
constexpr int xhalf_stride();

template <typename T, int L1, int L2, bool FULL>
__device__ __forceinline__ void fwd_half_rest(const X4Args<T>& a, cpx<T>* v, cpx<T>* line,
                                              cpx<T>* lds, int t, int q, int tid, int nthr, int c,
                                              int z, int y0, int nl) {
  using V = cpx<T>;
  constexpr int L = L1 * L2, R = L1 / 2, H = xhalf_stride<L>();
  if constexpr (!FULL && L1 >= 2) reg_fft_hz<T, L1, false>(v);
  else reg_fft<T, L1, false>(v);
  V x1[L1];
#pragma unroll
  for (int k1 = 0; k1 < L1; ++k1) {
    V x = v[bitrev<L1>(k1)];
    if (k1 > 0) x = cmul(x, a.tw4[k1 * L2 + t]);
    x1[k1] = x;
  }
  pin_regs<L1, T>(x1);
  V u[L1 / L2][L2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    // rows k1 of this half at local row k1 - h R (same swizzle as the
    // whole-line transpose)
#pragma unroll
    for (int k1 = h * R; k1 < (h + 1) * R; ++k1)
      line[(k1 - h * R) * L2 + (t ^ (k1 & (L2 - 1)))] = x1[k1];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < L1 / L2; ++i) {
      const int k1 = t + L2 * i;
      if ((k1 >= R) == (h == 1)) {
#pragma unroll
        for (int n2 = 0; n2 < L2; ++n2)
          u[i][n2] = line[(k1 - h * R) * L2 + (n2 ^ (k1 & (L2 - 1)))];
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < L1 / L2; ++i) pin_regs<L2, T>(u[i]);
#pragma unroll
  for (int i = 0; i < L1 / L2; ++i) reg_fft<T, L2, false>(u[i]);
#pragma unroll
  for (int i = 0; i < L1 / L2; ++i) pin_regs<L2, T>(u[i]);
  V* out = a.S1 + ((long)(c * a.nz + z) * a.Hx) * a.ldy + y0;
  const int sq = xsw<L>(q);
  const T hf = T(0.5);
  // spectrum half 0: bins [0, L/4) at their index, (3L/4, L) at k - L/2;
  // half 1: bins [L/4, 3L/4] at k - L/4
#pragma unroll
  for (int h = 0; h < 2; ++h) {
#pragma unroll
    for (int i = 0; i < L1 / L2; ++i)
#pragma unroll
      for (int k2 = 0; k2 < L2; ++k2) {
        const int k = t + L2 * i + L1 * k2;
        const bool mid = k >= L / 4 && k <= 3 * L / 4;
        if (mid == (h == 1)) {
          const int loc = h ? k - L / 4 : (k < L / 4 ? k : k - L / 2);
          line[loc ^ sq] = u[i][bitrev<L2>(k2)];
        }
      }
    __syncthreads();
    // this half's bins kx (and their partners L - kx), every line of the block
    const int kx0 = h ? L / 4 : 0, cnt = h ? L / 4 + 1 : L / 4;
    for (int idx = tid; idx < nl * cnt; idx += nthr) {
      const int qq = idx & (nl - 1), kx = kx0 + (idx >> a.lnl);
      const int kp = (L - kx) & (L - 1);
      const int lk = h ? kx - L / 4 : kx;
      const int lp = h ? kp - L / 4 : (kp < L / 4 ? kp : kp - L / 2);
      const V* lq = lds + qq * H;
      const V zk = lq[lk ^ xsw<L>(qq)];
      const V zm = lq[lp ^ xsw<L>(qq)];
      store2<T>(out + (long)kx * a.ldy + 2 * qq, cmk<T>(hf * (zk.x + zm.x), hf * (zk.y - zm.y)),
                cmk<T>(hf * (zk.y + zm.y), hf * (zm.x - zk.x)));
    }
    if (h == 0) __syncthreads();
  }
}

// LDS elements per line of the half-LDS x forward pass: half a line, plus
// one aligned group of 32 for the last element of the second spectrum half
// and the bank swizzle
template <int L>
constexpr int xhalf_stride() { return L / 2 + 32; }

// HALF (lines of 64 points or more): the step-1/step-3 transpose and the
// unpack each go through LDS in two halves of a line (rows k1 < L1/2, then
// the rest; spectrum bins k in [0, L/4) and (3L/4, L), then [L/4, 3L/4]),
// so a block holds half the LDS and twice as many blocks fit on a CU.
template <typename T, int L1, int L2, bool FULL, bool HALF = false>
__global__ __launch_bounds__(256) void k4_fftx_fwd(X4Args<T> a) {
  using V = cpx<T>;
  if (ctrl_stopped(a.ctrl)) return;
  constexpr int L = L1 * L2;
  extern __shared__ char smem_raw[];
  V* lds = reinterpret_cast<V*>(smem_raw);
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int t = tid % L2, q = tid / L2;
  const int c = blockIdx.z, z = blockIdx.y, y0 = blockIdx.x * a.ty;
  const int nl = a.ty >> 1;
  const long N = (long)a.nx * a.ny * a.nz;
  const gcptr<T> m = (gcptr<T>)stage_in(a.tbl, a.stage);
  const gcptr<T> m0 = m + (long)c * N + (long)z * a.ny * a.nx;
  const gcptr<T> m1 = m0 + 3 * N;
  const int ya = y0 + 2 * q, yb = ya + 1;
  V* line = lds + q * (HALF ? xhalf_stride<L>() : L);
  V v[L1];
  constexpr int NLOAD = (!FULL && L1 >= 2) ? L1 / 2 : L1;
  // rows ya, yb (clamped to row 0 past ny, column 0 past nx): every load is
  // unconditional so they all go out before the first wait
  const long ra = (long)(ya < a.ny ? ya : 0) * a.nx, rb = (long)(yb < a.ny ? yb : 0) * a.nx;
  T xa[NLOAD], xb[NLOAD];
#pragma unroll
  for (int n1 = 0; n1 < NLOAD; ++n1) {
    const int x = L2 * n1 + t;
    const int xc = x < a.nx ? x : 0;
    xa[n1] = a.ms0 * m0[ra + xc];
    xb[n1] = a.ms0 * m0[rb + xc];
  }
  if (a.nsub >= 2) {
#pragma unroll
    for (int n1 = 0; n1 < NLOAD; ++n1) {
      const int x = L2 * n1 + t;
      const int xc = x < a.nx ? x : 0;
      xa[n1] += a.ms1 * m1[ra + xc];
      xb[n1] += a.ms1 * m1[rb + xc];
    }
  }
  if (a.nsub == 3) {
    const gcptr<T> m2 = m1 + 3 * N;
#pragma unroll
    for (int n1 = 0; n1 < NLOAD; ++n1) {
      const int x = L2 * n1 + t;
      const int xc = x < a.nx ? x : 0;
      xa[n1] += a.ms2 * m2[ra + xc];
      xb[n1] += a.ms2 * m2[rb + xc];
    }
  }
#pragma unroll
  for (int n1 = 0; n1 < NLOAD; ++n1) {
    const bool inx = L2 * n1 + t < a.nx;
    v[n1] = cmk<T>(inx && ya < a.ny ? xa[n1] : T(0), inx && yb < a.ny ? xb[n1] : T(0));
  }
  if constexpr (HALF) {
    fwd_half_rest<T, L1, L2, FULL>(a, v, line, lds, t, q, tid, nthr, c, z, y0, nl);
    return;
  }
  fs_step1<T, L1, L2, false, !FULL>(v, line, a.tw4, t);
  __syncthreads();
  V u[L1 / L2][L2];
  fs_step3<T, L1, L2, false>(u, line, t);
  __syncthreads();
  const int sq = xsw<L>(q);
#pragma unroll
  for (int i = 0; i < L1 / L2; ++i)
#pragma unroll
    for (int k2 = 0; k2 < L2; ++k2) line[(t + L2 * i + L1 * k2) ^ sq] = u[i][bitrev<L2>(k2)];
  __syncthreads();
  // unpack the two real spectra and store them transposed (y contiguous,
  // rows 2qq and 2qq+1 as one 16-byte store for FP32)
  V* out = a.S1 + ((long)(c * a.nz + z) * a.Hx) * a.ldy + y0;
  auto unpack = [&](int qq, int kx) {
    const V zk = lds[qq * L + (kx ^ xsw<L>(qq))];
    const V zm = lds[qq * L + (((L - kx) & (L - 1)) ^ xsw<L>(qq))];
    const T h = T(0.5);
    store2<T>(out + (long)kx * a.ldy + 2 * qq, cmk<T>(h * (zk.x + zm.x), h * (zk.y - zm.y)),
              cmk<T>(h * (zk.y + zm.y), h * (zm.x - zk.x)));
  };
  // kx < Hx - 1 = L/2 spread evenly over the threads; the Nyquist bin rides
  // with kx = 0 (no extra, nearly empty round for the whole block)
  // (a one-cell axis, L = 1, has the single bin kx = 0)
  const int nh = a.Hx - 1;
  for (int idx = tid; idx < nl * (nh > 0 ? nh : 1); idx += nthr) {
    const int qq = idx & (nl - 1), kx = idx >> a.lnl;
    unpack(qq, kx);
    if (kx == 0 && nh > 0) unpack(qq, nh);
  }
}

template <typename T, int L1, int L2>
__global__ __launch_bounds__(256) void k4_fftx_inv(X4Args<T> a) {
  using V = cpx<T>;
  if (ctrl_stopped(a.ctrl)) return;
  constexpr int L = L1 * L2;
  extern __shared__ char smem_raw[];
  V* lds = reinterpret_cast<V*>(smem_raw);
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int t = tid % L2, q = tid / L2;
  const int c = blockIdx.z, z = blockIdx.y, y0 = blockIdx.x * a.ty;
  const int nl = a.ty >> 1;
  const V* in = a.S1 + ((long)(c * a.nz + z) * a.Hx) * a.ldy + y0;
  // spectrum pairs kx < Hx - 1 = L/2 of the block over its nl L2 threads:
  // L1/2 each, all loads unconditional (clamped to pair 0) and issued before
  // the first wait; the Nyquist pair rides with kx = 0 (threads tid < nl)
  constexpr int NI = L1 / 2;
  const int nh = a.Hx - 1;
  const int npair = nl * nh;
  V pa[NI > 0 ? NI : 1], pb[NI > 0 ? NI : 1], qa, qb;
#pragma unroll
  for (int j = 0; j < NI; ++j) {
    const int idx = tid + j * nthr;
    const int ic = idx < npair ? idx : 0;
    const int qq = ic & (nl - 1), kx = ic >> a.lnl;
    load2<T>(in + (long)kx * a.ldy + 2 * qq, pa[j], pb[j]);
  }
  const bool nyq = tid < nl;
  load2<T>(in + (long)nh * a.ldy + 2 * (nyq ? tid : 0), qa, qb);
#pragma unroll
  for (int j = 0; j < NI; ++j) {
    const int idx = tid + j * nthr;
    if (idx < npair) {
      const int qq = idx & (nl - 1), kx = idx >> a.lnl;
      const V xa = pa[j], xb = pb[j];
      lds[qq * L + (kx ^ xsw<L>(qq))] = cmk<T>(xa.x - xb.y, xa.y + xb.x);
      if (kx > 0 && 2 * kx < L)
        lds[qq * L + ((L - kx) ^ xsw<L>(qq))] = cmk<T>(xa.x + xb.y, xb.x - xa.y);
    }
  }
  if (nyq) lds[tid * L + (nh ^ xsw<L>(tid))] = cmk<T>(qa.x - qb.y, qa.y + qb.x);
  __syncthreads();
  V* line = lds + q * L;
  V v[L1];
#pragma unroll
  for (int n1 = 0; n1 < L1; ++n1) v[n1] = line[(L2 * n1 + t) ^ xsw<L>(q)];
  __syncthreads();
  fs_step1<T, L1, L2, true>(v, line, a.tw4, t);
  __syncthreads();
  V u[L1 / L2][L2];
  fs_step3<T, L1, L2, true>(u, line, t);
  const long N = (long)a.nx * a.ny * a.nz;
  T* out = a.Bd + (long)c * N + (long)z * a.ny * a.nx;
  const int ya = y0 + 2 * q;
#pragma unroll
  for (int i = 0; i < L1 / L2; ++i)
#pragma unroll
    for (int k2 = 0; k2 < L2; ++k2) {
      const int x = t + L2 * i + L1 * k2;
      if (x < a.nx) {
        const cpx<T> r = u[i][bitrev<L2>(k2)];
        if (ya < a.ny) out[(long)ya * a.nx + x] = r.x;
        if (ya + 1 < a.ny) out[(long)(ya + 1) * a.nx + x] = r.y;
      }
    }
}

// ---------------------------------------------- 2-D fused y + multiply --
template <typename T, int L1, int L2, bool FULL>
__global__ __launch_bounds__(256) void k4_ffty_mul2d(M4Args<T> a) {
  using V = cpx<T>;
  if (ctrl_stopped(a.ctrl)) return;
  constexpr int L = L1 * L2;
  extern __shared__ char smem_raw[];
  V* lds = reinterpret_cast<V*>(smem_raw);
  const int t = threadIdx.x % L2, ln = threadIdx.x / L2;
  const int c = ln / a.nk, j = ln - c * a.nk;
  const int kx = blockIdx.x * a.nk + j;
  const bool valid = kx < a.Hx;
  V* line = lds + ln * L;
  V* io = a.S1 + ((long)c * a.Hx + kx) * a.ldy;
  V v[L1];
  constexpr int NLOAD = (!FULL && L1 >= 2) ? L1 / 2 : L1;
#pragma unroll
  for (int n1 = 0; n1 < NLOAD; ++n1) {
    const int y = L2 * n1 + t;
    v[n1] = (valid && y < a.ny) ? io[y] : cmk<T>(0, 0);
  }
  fs_step1<T, L1, L2, false, !FULL>(v, line, a.tw4, t);
  __syncthreads();
  V u[L1 / L2][L2];
  fs_step3<T, L1, L2, false>(u, line, t);
  __syncthreads();
#pragma unroll
  for (int i = 0; i < L1 / L2; ++i)
#pragma unroll
    for (int k2 = 0; k2 < L2; ++k2) line[t + L2 * i + L1 * k2] = u[i][bitrev<L2>(k2)];
  __syncthreads();
  // inverse step 1 loads B_c = sum_j K_cj M_j at ky = L2 n1 + t
  const V* lx = lds + (0 * a.nk + j) * L;
  const V* ly = lds + (1 * a.nk + j) * L;
  const V* lz = lds + (2 * a.nk + j) * L;
  const long ks = (long)a.Hx * a.Hy;
  // row c of the 2-D kernel (K_xz = K_yz = 0):  c = 0: (xx, sy xy, 0),
  // c = 1: (sy xy, yy, 0),  c = 2: (0, 0, zz).  Both kernel values of every
  // ky are loaded first (kx clamped for the idle columns past Hx), so the
  // loads go out back to back.
  const T* kc = a.K + (long)(valid ? kx : 0) * a.Hy;
  const long oa = (c == 0 ? 0 : c == 1 ? 3 : 2) * ks, ob = (c == 0 ? 3 : c == 1 ? 1 : 2) * ks;
  T ka[L1], kb[L1];
#pragma unroll
  for (int n1 = 0; n1 < L1; ++n1) {
    const int ky = L2 * n1 + t;
    const int kyo = ky <= L / 2 ? ky : L - ky;
    ka[n1] = kc[oa + kyo];
    kb[n1] = kc[ob + kyo];
  }
#pragma unroll
  for (int n1 = 0; n1 < L1; ++n1) {
    const int ky = L2 * n1 + t;
    const T sy = ky <= L / 2 ? T(1) : T(-1);
    const V m1 = c == 2 ? lz[ky] : lx[ky];
    const V m2 = ly[ky];
    const T f1 = c == 1 ? sy * ka[n1] : ka[n1];
    const T f2 = c == 2 ? T(0) : (c == 0 ? sy * kb[n1] : kb[n1]);
    v[n1] = valid ? cmk<T>(f1 * m1.x + f2 * m2.x, f1 * m1.y + f2 * m2.y) : cmk<T>(0, 0);
  }
  __syncthreads();
  fs_step1<T, L1, L2, true>(v, line, a.tw4, t);
  __syncthreads();
  fs_step3<T, L1, L2, true>(u, line, t);
  if (valid) {
#pragma unroll
    for (int i = 0; i < L1 / L2; ++i)
#pragma unroll
      for (int k2 = 0; k2 < L2; ++k2) {
        const int y = t + L2 * i + L1 * k2;
        if (y < a.ny) io[y] = u[i][bitrev<L2>(k2)];
      }
  }
}

// ------------------------------------------ 3-D z columns + multiply ----
// The value that lane (lane ^ X) of the same quad holds, X = 1, 2 or 3 (DPP
// quad permutations [1,0,3,2], [2,3,0,1] and [3,2,1,0]; no LDS traffic).
template <int X>
__device__ __forceinline__ int quad_xor_i(int v) {
  static_assert(X >= 1 && X <= 3, "quad lane mask");
  return __builtin_amdgcn_update_dpp(0, v, X == 1 ? 0xB1 : (X == 2 ? 0x4E : 0x1B), 0xF, 0xF,
                                     false);
}
template <int X>
__device__ __forceinline__ float quad_xor(float v) {
  return __int_as_float(quad_xor_i<X>(__float_as_int(v)));
}
template <int X>
__device__ __forceinline__ double quad_xor(double v) {
  return __hiloint2double(quad_xor_i<X>(__double2hiint(v)), quad_xor_i<X>(__double2loint(v)));
}
template <int X, typename T>
__device__ __forceinline__ cpx<T> quad_xor_c(cpx<T> v) {
  return cmk<T>(quad_xor<X>(v.x), quad_xor<X>(v.y));
}

// f(integral_constant<int, I>) for I = B .. E-1, unrolled at compile time
template <int I, int E, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (I < E) {
    f(std::integral_constant<int, I>{});
    static_for<I + 1, E>(f);
  }
}

// exp(-/+ 2 pi i n q / P) for compile-time n, P and a lane index q < Q
template <typename T, int N, int P, int Q, bool INV>
__device__ __forceinline__ cpx<T> lane_root(int q) {
  cpx<T> w = cmk<T>(T(1), T(0));
  if constexpr (Q >= 2)
    if (q == 1) w = root<T, N, P, INV>();
  if constexpr (Q >= 4) {
    if (q == 2) w = root<T, 2 * N, P, INV>();
    if (q == 3) w = root<T, 3 * N, P, INV>();
  }
  return w;
}

// exp(-2 pi i n t / P) with n = N0 + q and t = q ^ D, for the lane index q < Q
template <typename T, int P, int Q, int D, int N0>
__device__ __forceinline__ cpx<T> split_root(int q) {
  cpx<T> w = root<T, (N0 * D) % P, P, false>();
  if constexpr (Q >= 2)
    if (q == 1) w = root<T, ((N0 + 1) * (1 ^ D)) % P, P, false>();
  if constexpr (Q >= 4) {
    if (q == 2) w = root<T, ((N0 + 2) * (2 ^ D)) % P, P, false>();
    if (q == 3) w = root<T, ((N0 + 3) * (3 ^ D)) % P, P, false>();
  }
  return w;
}

// Forward input of the Q lanes of a column with the loads shared: lane t
// needs its twisted, folded column y_t(r) = sum over n = r (mod R) of
// x(n) w^(n t), R = PZ/Q.  When Q divides R every plane n of a residue r
// lies in lane r mod Q, so lane q loads only the planes n = Q i + q, forms
// for each lane t = q ^ D of the quad the terms of t's residues r = q + Q j
// that its planes carry, and the terms reach t by the quad permutation ^D.
// The sums and twiddles are those of loading every plane in every lane, at
// 1/Q of the loads and of the registers they occupy.
template <typename T, int PZ, int Q>
__device__ __forceinline__ void zcol_load_split(const cpx<T>* col, long zs, long cs, int nz,
                                                int q, cpx<T>* vx, cpx<T>* vy, cpx<T>* vz) {
  using V = cpx<T>;
  constexpr int R = PZ / Q, NH = PZ / 2, NL = NH / Q, J = R / Q, K = NH / R;
  static_assert(Q > 1 && R % Q == 0 && NL >= 1 && K >= 1, "shared column loads");
  V l[3][NL];
#pragma unroll
  for (int i = 0; i < NL; ++i) {
    const int n = Q * i + q;
    const long off = (long)(n < nz ? n : 0) * zs;
    l[0][i] = ntload(col + off);
    l[1][i] = ntload(col + cs + off);
    l[2][i] = ntload(col + 2 * cs + off);
  }
#pragma unroll
  for (int i = 0; i < NL; ++i)
    if (Q * i + q >= nz) l[0][i] = l[1][i] = l[2][i] = cmk<T>(0, 0);
  V in[3][Q][J];
  static_for<0, Q>([&](auto dc) {
    constexpr int D = decltype(dc)::value;
    static_for<0, J>([&](auto jc) {
      constexpr int j = decltype(jc)::value;
      V acc[3] = {cmk<T>(0, 0), cmk<T>(0, 0), cmk<T>(0, 0)};
      static_for<0, K>([&](auto kc) {
        constexpr int k = decltype(kc)::value;
        const V w = split_root<T, PZ, Q, D, Q * j + R * k>(q);
#pragma unroll
        for (int c = 0; c < 3; ++c) acc[c] = cadd(acc[c], cmul(l[c][j + J * k], w));
      });
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        if constexpr (D == 0) in[c][D][j] = acc[c];
        else in[c][D][j] = quad_xor_c<D, T>(acc[c]);
      }
    });
  });
  // residue r = p + Q j came from lane p through the permutation ^(p ^ q)
#pragma unroll
  for (int p = 0; p < Q; ++p) {
    const int D = p ^ q;
#pragma unroll
    for (int j = 0; j < J; ++j) {
      V o[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        o[c] = in[c][0][j];
        if (D == 1) o[c] = in[c][1][j];
        if constexpr (Q >= 4) {
          if (D == 2) o[c] = in[c][2][j];
          if (D == 3) o[c] = in[c][3][j];
        }
      }
      vx[p + Q * j] = o[0];
      vy[p + Q * j] = o[1];
      vz[p + Q * j] = o[2];
    }
  }
}

// one complex value through a global-typed pointer (a global, not flat,
// store), component by component: the vector type's assignment does not
// take an address-space-qualified destination
template <typename T>
__device__ __forceinline__ void gstore(gptr<cpx<T>> p, cpx<T> v) {
  const gptr<T> q = (gptr<T>)p;
  q[0] = v.x;
  q[1] = v.y;
}

// Inverse transform of one component held by the Q lanes of a column and
// store of the first nz planes.  Lane q holds B(kz = Q j + q) at register
// bitrev<R>(j); with R = PZ/Q,
//   b(n) = sum_q w^(-n q) IFFT_R(B(Q j + q))(n mod R),
// so each lane forms its term for n < PZ/2 and the Q lanes sum them with a
// recursive-halving exchange that leaves lane q owning PZ/(2Q) planes.
// Plain stores: the y inverse pass reads these planes next, and part of
// them is still in the Infinity Cache when it does.
template <typename T, int PZ, int Q>
__device__ __forceinline__ void zcol_inverse_store(cpx<T>* v, gptr<cpx<T>> col, long zs, int nz,
                                                   int q) {
  using V = cpx<T>;
  constexpr int R = PZ / Q, NH = PZ / 2;
  V t[R];
#pragma unroll
  for (int k = 0; k < R; ++k) t[k] = v[bitrev<R>(k)];
  reg_fft<T, R, true>(t);
  if constexpr (Q == 1) {
#pragma unroll
    for (int z = 0; z < NH; ++z)
      if (z < nz) gstore<T>(col + z * zs, t[bitrev<PZ>(z)]);
  } else {
    V c[NH];
    static_for<0, NH>([&](auto nc) {
      constexpr int n = decltype(nc)::value;
      const V x = t[bitrev<R>(n % R)];
      if constexpr (n == 0) c[n] = x;
      else c[n] = cmul(x, lane_root<T, n, PZ, Q, true>(q));
    });
    int base = 0;
    if constexpr (Q == 4) {
      const bool hi = (q & 2) != 0;
#pragma unroll
      for (int i = 0; i < NH / 2; ++i) {
        const V send = hi ? c[i] : c[i + NH / 2];
        const V keep = hi ? c[i + NH / 2] : c[i];
        c[i] = cadd(keep, quad_xor_c<2, T>(send));
      }
      base += hi ? NH / 2 : 0;
    }
    constexpr int S = 2 * NH / Q;  // planes held before the last exchange
    const bool hi = (q & 1) != 0;
#pragma unroll
    for (int i = 0; i < S / 2; ++i) {
      const V send = hi ? c[i] : c[i + S / 2];
      const V keep = hi ? c[i + S / 2] : c[i];
      c[i] = cadd(keep, quad_xor_c<1, T>(send));
    }
    base += hi ? S / 2 : 0;
#pragma unroll
    for (int i = 0; i < S / 2; ++i)
      if (base + i < nz) gstore<T>(col + (base + i) * zs, c[i]);
  }
}

// B(kz) = K(kz) M(kz) for the spectra of one column, held at bit-reversed
// register positions; kv(c, j, kzo) is kernel component c (xx, yy, zz, xy,
// xz, yz) at the mirrored plane kzo of lane q's register j.  The stored
// octant is mirrored to the full spectrum: the diagonal components are even
// in every wave number, an off-diagonal one is odd in each of the two wave
// numbers it pairs (sy past Py/2, sz past Pz/2; kx is never mirrored).
template <typename T, int PZ, int Q, typename KV>
__device__ __forceinline__ void zcol_kmul(cpx<T>* vx, cpx<T>* vy, cpx<T>* vz, int q, T sy,
                                          KV&& kv) {
  constexpr int R = PZ / Q;
#pragma unroll
  for (int j = 0; j < R; ++j) {
    const int kz = Q * j + q;
    const int kzo = kz <= PZ / 2 ? kz : PZ - kz;
    const T sz = kz <= PZ / 2 ? T(1) : T(-1);
    T k6[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) k6[c] = kv(c, j, kzo);
    const T kxx = k6[0], kyy = k6[1], kzz = k6[2];
    const T kxy = sy * k6[3], kxz = sz * k6[4], kyz = sy * sz * k6[5];
    const int r = bitrev<R>(j);
    const cpx<T> mx = vx[r], my = vy[r], mz = vz[r];
    vx[r] = cmk<T>(kxx * mx.x + kxy * my.x + kxz * mz.x, kxx * mx.y + kxy * my.y + kxz * mz.y);
    vy[r] = cmk<T>(kxy * mx.x + kyy * my.x + kyz * mz.x, kxy * mx.y + kyy * my.y + kyz * mz.y);
    vz[r] = cmk<T>(kxz * mx.x + kyz * my.x + kzz * mz.x, kxz * mx.y + kyz * my.y + kzz * mz.y);
  }
}

// Asynchronous copy of one 32-bit word per lane from global memory into LDS
// (the lanes' words land at consecutive addresses from wave-uniform dst): the
// data occupies no registers while in flight and completes with vmcnt.
__device__ __forceinline__ void lds_dma_b32(const float* src, float* dst) {
  __builtin_amdgcn_global_load_lds((__attribute__((address_space(1))) void*)const_cast<float*>(src),
                                   (__attribute__((address_space(3))) void*)dst, 4, 0, 0);
}

// K rows a lane of the register z pass reads: with one lane per column the
// PZ/2 + 1 distinct planes kzo of the mirrored spectrum, else one per
// register j (lane q's kz = Q j + q).
template <int PZ, int Q>
constexpr int zk_rows() { return Q == 1 ? PZ / 2 + 1 : PZ / Q; }


// Q adjacent lanes (Q = 1, 2 or 4, within one quad) carry the three
// components of one (kx, ky) column through forward FFT, kernel multiply and
// inverse FFT in registers: no LDS and no barriers, so the pass streams like
// a copy.  Lane q computes the spectrum at kz = q mod Q: it twists the data by
// w^(n q), folds it modulo R = PZ/Q and takes an R-point transform, so more
// lanes per column mean fewer registers per lane.  Blocks are ordered so that
// all ky tiles of one kx run back to back on one XCD, which keeps that kx
// slice of the kernel (read for ky and its mirror Py - ky) in the XCD's L2.
// KL: the lane's 6 zk_rows kernel values are copied into the wave's LDS
// slice right behind the column loads, so both latencies overlap and the
// multiply reads LDS instead of waiting on a second round of loads after the
// forward transforms (one wave per SIMD leaves nothing else to hide it).
template <typename T, int PZ, int Q, bool KL>
__device__ __forceinline__ void fftz_mul_body(const Z4Args<T>& a) {
  using V = cpx<T>;
  constexpr int R = PZ / Q, NH = PZ / 2;
  static_assert(zreg_ok((int)sizeof(T), PZ, Q), "lanes per column");
  static_assert(!KL || sizeof(T) == 4, "LDS-staged kernel values are 32-bit words");
  if (ctrl_stopped(a.ctrl)) return;
  const int cpb = blockDim.x / Q;
  const int ntile = (a.Py + cpb - 1) / cpb;
  const int w = xcd_remap(blockIdx.x, a.nb_pad);
  if (w >= ntile * a.Hx) return;
  const int q = threadIdx.x % Q;
  const int kx = w / ntile, ky = (w - kx * ntile) * cpb + threadIdx.x / Q;
  if (ky >= a.Py) return;
  const long zs = (long)a.Hx * a.Py;
  const long cs = (long)a.nz * zs;
  V* col = a.S2 + (long)kx * a.Py + ky;
  V vx[R], vy[R], vz[R];
  // nz <= PZ/2 for every power-of-two pad, so the upper half is zero
  if constexpr (Q > 1 && (PZ / Q) % Q == 0) {
    zcol_load_split<T, PZ, Q>(col, zs, cs, a.nz, q, vx, vy, vz);
  } else {
    // all planes are loaded first (a plain unrolled loop keeps the loads
    // back to back), then lane q twists them by w^(n q) and folds mod R
    V lx[NH], ly[NH], lz[NH];
#pragma unroll
    for (int n = 0; n < NH; ++n) {
      const bool in = n < a.nz;
      lx[n] = in ? ntload(col + n * zs) : cmk<T>(0, 0);
      ly[n] = in ? ntload(col + cs + n * zs) : cmk<T>(0, 0);
      lz[n] = in ? ntload(col + 2 * cs + n * zs) : cmk<T>(0, 0);
    }
    static_for<0, NH>([&](auto nc) {
      constexpr int n = decltype(nc)::value;
      V x = lx[n], y = ly[n], z = lz[n];
      if constexpr (Q > 1 && n > 0) {
        const V wq = lane_root<T, n, PZ, Q, false>(q);
        x = cmul(x, wq);
        y = cmul(y, wq);
        z = cmul(z, wq);
      }
      if constexpr (n < R) {
        vx[n] = x; vy[n] = y; vz[n] = z;
      } else {
        vx[n % R] = cadd(vx[n % R], x); vy[n % R] = cadd(vy[n % R], y);
        vz[n % R] = cadd(vz[n % R], z);
      }
    });
  }
  const int kyo = ky <= a.Py / 2 ? ky : a.Py - ky;
  const T sy = ky <= a.Py / 2 ? T(1) : T(-1);
  const long ks = (long)a.Hz * a.Hx * a.Hy;
  const T* K = a.K + (long)kx * a.Hy + kyo;
  const long kzs = (long)a.Hx * a.Hy;
  constexpr int NJ = zk_rows<PZ, Q>();
  [[maybe_unused]] T* kw = nullptr;
  if constexpr (KL) {
    extern __shared__ char smem_raw[];
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);  // uniform: M0 is scalar
    kw = reinterpret_cast<T*>(smem_raw) + wv * (6 * NJ * 64);
#pragma unroll
    for (int c = 0; c < 6; ++c)
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        int kzo = j;
        if constexpr (Q > 1) {
          const int kz = Q * j + q;
          kzo = kz <= PZ / 2 ? kz : PZ - kz;
        }
        lds_dma_b32(K + c * ks + kzo * kzs, kw + (c * NJ + j) * 64);
      }
  }
  if constexpr (Q == 1) {
    reg_fft_hz<T, PZ, false>(vx);
    reg_fft_hz<T, PZ, false>(vy);
    reg_fft_hz<T, PZ, false>(vz);
  } else {
    reg_fft<T, R, false>(vx);
    reg_fft<T, R, false>(vy);
    reg_fft<T, R, false>(vz);
  }
  pin_regs<R, T>(vx);
  pin_regs<R, T>(vy);
  pin_regs<R, T>(vz);
  const int lane = threadIdx.x & 63;
  // the LDS copies complete with the vector memory counter (vmcnt 0)
  if constexpr (KL) __builtin_amdgcn_s_waitcnt(0x0F70);
  zcol_kmul<T, PZ, Q>(vx, vy, vz, q, sy, [&](int c, int j, int kzo) {
    if constexpr (KL) return kw[(c * NJ + (Q == 1 ? kzo : j)) * 64 + lane];
    else return K[kzo * kzs + c * ks];
  });
  pin_regs<R, T>(vx);
  pin_regs<R, T>(vy);
  pin_regs<R, T>(vz);
  // the store addresses are formed anew, not kept in registers from the
  // loads (through a global-typed pointer: global, not flat, stores)
  gptr<V> gcol = (gptr<V>)col;
  asm volatile("" : "+v"(gcol));
  zcol_inverse_store<T, PZ, Q>(vx, gcol, zs, a.nz, q);
  zcol_inverse_store<T, PZ, Q>(vy, gcol + cs, zs, a.nz, q);
  zcol_inverse_store<T, PZ, Q>(vz, gcol + 2 * cs, zs, a.nz, q);
}

// W > 1: ask the register allocator for at least W waves per SIMD
template <typename T, int PZ, int Q, int W>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(W))) void k4_fftz_mul_w(
    Z4Args<T> a) {
  fftz_mul_body<T, PZ, Q, false>(a);
}
template <typename T, int PZ, int Q>
__global__ __launch_bounds__(256) void k4_fftz_mul(Z4Args<T> a) {
  fftz_mul_body<T, PZ, Q, false>(a);
}
template <typename T, int PZ, int Q>
__global__ __launch_bounds__(256) void k4_fftz_mul_kl(Z4Args<T> a) {
  fftz_mul_body<T, PZ, Q, true>(a);
}

// ------------------------------------------------------------ dispatch --
#define MMP_L_CASES(X) \
  X(1) X(2) X(4) X(8) X(16) X(32) X(64) X(128) X(256) X(512) X(1024) X(2048) X(4096)

template <typename T, int L>
static void ly(bool inv, bool full, dim3 g, int thr, size_t lds, hipStream_t st,
               const Y4Args<T>& a) {
  constexpr int L1 = Split<L>::L1, L2 = Split<L>::L2;
  if (inv) hipLaunchKernelGGL((k4_ffty<T, L1, L2, true, false>), g, dim3(thr), lds, st, a);
  else if (full) hipLaunchKernelGGL((k4_ffty<T, L1, L2, false, true>), g, dim3(thr), lds, st, a);
  else hipLaunchKernelGGL((k4_ffty<T, L1, L2, false, false>), g, dim3(thr), lds, st, a);
}

template <typename T>
void launch_y4(int L, bool inv, bool full, dim3 g, int thr, size_t lds, hipStream_t st,
               const Y4Args<T>& a) {
  switch (L) {
#define X(n) case n: ly<T, n>(inv, full, g, thr, lds, st, a); break;
    MMP_L_CASES(X)
#undef X
  }
}

template <typename T, int L>
static void lx(bool inv, bool full, dim3 g, int thr, size_t lds, hipStream_t st,
               const X4Args<T>& a) {
  constexpr int L1 = Split<L>::L1, L2 = Split<L>::L2;
  // half-LDS forward pass for 32-bit values (x4_lds_bytes); 64-bit lines
  // would hold more registers than the LDS saving gains
  constexpr bool H = L >= 64 && sizeof(T) == 4;
  if (inv) hipLaunchKernelGGL((k4_fftx_inv<T, L1, L2>), g, dim3(thr), lds, st, a);
  else if (full) hipLaunchKernelGGL((k4_fftx_fwd<T, L1, L2, true, H>), g, dim3(thr), lds, st, a);
  else hipLaunchKernelGGL((k4_fftx_fwd<T, L1, L2, false, H>), g, dim3(thr), lds, st, a);
}

template <typename T>
void launch_x4(int L, bool inv, bool full, dim3 g, int thr, size_t lds, hipStream_t st,
               const X4Args<T>& a) {
  switch (L) {
#define X(n) case n: lx<T, n>(inv, full, g, thr, lds, st, a); break;
    MMP_L_CASES(X)
#undef X
  }
}

template <typename T, int L>
static void lm(bool full, dim3 g, int thr, size_t lds, hipStream_t st, const M4Args<T>& a) {
  constexpr int L1 = Split<L>::L1, L2 = Split<L>::L2;
  if (full) hipLaunchKernelGGL((k4_ffty_mul2d<T, L1, L2, true>), g, dim3(thr), lds, st, a);
  else hipLaunchKernelGGL((k4_ffty_mul2d<T, L1, L2, false>), g, dim3(thr), lds, st, a);
}

template <typename T>
void launch_m4(int L, bool full, dim3 g, int thr, size_t lds, hipStream_t st,
               const M4Args<T>& a) {
  switch (L) {
#define X(n) case n: lm<T, n>(full, g, thr, lds, st, a); break;
    MMP_L_CASES(X)
#undef X
  }
}

template <typename T, int PZ, int Q, int W>
static bool lzw(int q, int w, int mode, dim3 g, int thr, hipStream_t st, const Z4Args<T>& a) {
  if constexpr (zreg_waves_ok((int)sizeof(T), PZ, Q, W)) {
    if (q == Q && w == W) {
      if constexpr (W == 1 && sizeof(T) == 4) {
        if (mode == 1) {
          hipLaunchKernelGGL((k4_fftz_mul_kl<T, PZ, Q>), g, dim3(thr),
                             (size_t)zk_lds_bytes(PZ, Q, thr), st, a);
          return true;
        }
      }
      if constexpr (W == 1)
        hipLaunchKernelGGL((k4_fftz_mul<T, PZ, Q>), g, dim3(thr), 0, st, a);
      else
        hipLaunchKernelGGL((k4_fftz_mul_w<T, PZ, Q, W>), g, dim3(thr), 0, st, a);
      return true;
    }
  }
  return false;
}

template <typename T, int PZ>
static void lz(int q, int w, int mode, dim3 g, int thr, hipStream_t st, const Z4Args<T>& a) {
  (void)(lzw<T, PZ, 1, 1>(q, w, mode, g, thr, st, a) || lzw<T, PZ, 1, 2>(q, w, mode, g, thr, st, a) ||
         lzw<T, PZ, 1, 4>(q, w, mode, g, thr, st, a) || lzw<T, PZ, 2, 1>(q, w, mode, g, thr, st, a) ||
         lzw<T, PZ, 2, 2>(q, w, mode, g, thr, st, a) || lzw<T, PZ, 2, 4>(q, w, mode, g, thr, st, a) ||
         lzw<T, PZ, 4, 1>(q, w, mode, g, thr, st, a) || lzw<T, PZ, 4, 2>(q, w, mode, g, thr, st, a) ||
         lzw<T, PZ, 4, 4>(q, w, mode, g, thr, st, a));
}

// The plan admits only (PZ, q, w) with zreg_waves_ok, so a launch is made.
template <typename T>
void launch_z4(int PZ, int q, int w, int mode, dim3 g, int thr, hipStream_t st,
               const Z4Args<T>& a) {
  switch (PZ) {
    case 2: lz<T, 2>(q, w, mode, g, thr, st, a); break;
    case 4: lz<T, 4>(q, w, mode, g, thr, st, a); break;
    case 8: lz<T, 8>(q, w, mode, g, thr, st, a); break;
    case 16: lz<T, 16>(q, w, mode, g, thr, st, a); break;
    case 32: lz<T, 32>(q, w, mode, g, thr, st, a); break;
    case 64: lz<T, 64>(q, w, mode, g, thr, st, a); break;
  }
}

#define INST(T)                                                                              \
  template void launch_y4<T>(int, bool, bool, dim3, int, size_t, hipStream_t,              \
                             const Y4Args<T>&);                                             \
  template void launch_x4<T>(int, bool, bool, dim3, int, size_t, hipStream_t,              \
                             const X4Args<T>&);                                             \
  template void launch_m4<T>(int, bool, dim3, int, size_t, hipStream_t, const M4Args<T>&);  \
  template void launch_z4<T>(int, int, int, int, dim3, int, hipStream_t, const Z4Args<T>&);
INST(float)
INST(double)

}  // namespace mmp
