// LDS-resident Stockham FFT engine (mixed radix 2/3/4/5/7/8) for gfx950.
//
// A work-group holds `nlines` lines of length L in LDS (line l starts at
// buf + l*ls) and transforms them in place: every stage loads each
// butterfly's inputs into registers, synchronises, and writes the autosorted
// outputs, so no second LDS buffer is needed.  Twiddles w^j = exp(-2 pi i
// j/L) come from an FP64-built table (indexes are exact integers, so no
// run-time trig in the passes); the kernels copy it into LDS beside the
// lines when it fits, so every stage reads it at LDS latency, and each
// thread issues the loads of all its butterflies of a stage before the
// first product.  The caller guarantees
// nlines*L <= kMaxE * blockDim.x, which bounds the butterflies per thread.
#pragma once

#include "common.h"

namespace mmp {

constexpr int kMaxE = 16;  // elements per thread per stage (register budget)

// Radix plan packed in one integer (4 bits per stage, first stage in the low
// bits) so kernels decode it with scalar shifts instead of indexing an array
// (which would put the argument struct in private memory).
struct Rad {
  int n;
  uint64_t code;
};

inline Rad make_rad(const int* r, int n) {
  Rad d;
  d.n = n;
  d.code = 0;
  for (int i = 0; i < n; ++i) d.code |= (uint64_t)r[i] << (4 * i);
  return d;
}

// cos/sin(2 pi j / R) for the odd radices, as exact-to-double literals
template <int R> struct RootTable;
template <> struct RootTable<3> {
  static constexpr double c[3] = {1.0, -0.5, -0.5};
  static constexpr double s[3] = {0.0, 0.86602540378443864676, -0.86602540378443864676};
};
template <> struct RootTable<5> {
  static constexpr double c[5] = {1.0, 0.30901699437494742410, -0.80901699437494742410,
                                  -0.80901699437494742410, 0.30901699437494742410};
  static constexpr double s[5] = {0.0, 0.95105651629515357212, 0.58778525229247312917,
                                  -0.58778525229247312917, -0.95105651629515357212};
};
template <> struct RootTable<7> {
  static constexpr double c[7] = {1.0, 0.62348980185873353053, -0.22252093395631440429,
                                  -0.90096886790241912624, -0.90096886790241912624,
                                  -0.22252093395631440429, 0.62348980185873353053};
  static constexpr double s[7] = {0.0, 0.78183148246802980871, 0.97492791218182360702,
                                  0.43388373911755812048, -0.43388373911755812048,
                                  -0.97492791218182360702, -0.78183148246802980871};
};

// In-register DFT of size R; forward uses exp(-2 pi i rk/R).
template <typename T, int R, bool INV>
__device__ __forceinline__ void dft_small(cpx<T>* v) {
  using V = cpx<T>;
  if constexpr (R == 2) {
    V a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  } else if constexpr (R == 4) {
    V s02 = cadd(v[0], v[2]), d02 = csub(v[0], v[2]);
    V s13 = cadd(v[1], v[3]), d13 = csub(v[1], v[3]);
    // forward: y1 = d02 - i d13, y3 = d02 + i d13
    V jd = INV ? cmk<T>(-d13.y, d13.x) : cmk<T>(d13.y, -d13.x);  // (+/-) i*d13
    v[0] = cadd(s02, s13);
    v[2] = csub(s02, s13);
    v[1] = cadd(d02, jd);
    v[3] = csub(d02, jd);
  } else if constexpr (R == 8) {
    const T h = T(0.70710678118654752440);
    V a[4], b[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      a[r] = cadd(v[r], v[r + 4]);
      b[r] = csub(v[r], v[r + 4]);
    }
    // b_r *= w8^r, w8 = exp(-/+ i pi/4)
    if (!INV) {
      b[1] = cmk<T>(h * (b[1].x + b[1].y), h * (b[1].y - b[1].x));
      b[2] = cmk<T>(b[2].y, -b[2].x);
      b[3] = cmk<T>(h * (b[3].y - b[3].x), -h * (b[3].x + b[3].y));
    } else {
      b[1] = cmk<T>(h * (b[1].x - b[1].y), h * (b[1].y + b[1].x));
      b[2] = cmk<T>(-b[2].y, b[2].x);
      b[3] = cmk<T>(-h * (b[3].x + b[3].y), h * (b[3].x - b[3].y));
    }
    dft_small<T, 4, INV>(a);
    dft_small<T, 4, INV>(b);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      v[2 * k] = a[k];
      v[2 * k + 1] = b[k];
    }
  } else {
    V in[R];
#pragma unroll
    for (int r = 0; r < R; ++r) in[r] = v[r];
#pragma unroll
    for (int k = 0; k < R; ++k) {
      V acc = in[0];
#pragma unroll
      for (int r = 1; r < R; ++r) {
        const int j = (r * k) % R;
        const T c = T(RootTable<R>::c[j]);
        const T s = INV ? T(RootTable<R>::s[j]) : T(-RootTable<R>::s[j]);
        acc.x += in[r].x * c - in[r].y * s;
        acc.y += in[r].x * s + in[r].y * c;
      }
      v[k] = acc;
    }
  }
}

template <typename T, int R, bool INV>
__device__ __forceinline__ void fft_stage(cpx<T>* buf, const cpx<T>* __restrict__ tw, int L,
                                          int nlines, int ls, int Ns, int tid, int nthr) {
  using V = cpx<T>;
  constexpr int MAXB = (kMaxE + R - 1) / R;
  const int Lr = L / R;
  const int total = nlines * Lr;
  const int tstride = Lr / Ns;  // = L / (Ns * R)
  // the loads of all of a thread's butterflies (LDS values and twiddle
  // table entries) are issued before the first twiddle product, so they
  // overlap instead of each butterfly waiting for its own
  V v[MAXB][R];
  V tt[MAXB][R];
#pragma unroll
  for (int q = 0; q < MAXB; ++q) {
    const int w = tid + q * nthr;
    if (w < total) {
      const int line = w / Lr;
      const int j = w - line * Lr;
      const int k = j % Ns;
      const V* b = buf + line * ls;
#pragma unroll
      for (int r = 0; r < R; ++r) v[q][r] = b[j + r * Lr];
      if (Ns > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) tt[q][r] = tw[r * k * tstride];
      }
    }
  }
  if (Ns > 1) {
#pragma unroll
    for (int q = 0; q < MAXB; ++q) {
      if (tid + q * nthr < total) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          V t = tt[q][r];
          if (INV) t.y = -t.y;
          v[q][r] = cmul(v[q][r], t);
        }
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < MAXB; ++q) {
    const int w = tid + q * nthr;
    if (w < total) {
      const int line = w / Lr;
      const int j = w - line * Lr;
      const int k = j % Ns;
      dft_small<T, R, INV>(v[q]);
      V* b = buf + line * ls;
      const int base = (j / Ns) * Ns * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) b[base + r * Ns] = v[q][r];
    }
  }
  __syncthreads();
}

// P2: the plan has only radices 8/4/2 (power-of-two length); the odd-radix
// stages are then not compiled into the kernel, which keeps its register
// footprint small enough to avoid spilling.
template <typename T, bool INV, bool P2>
__device__ __forceinline__ void lds_fft(cpx<T>* buf, const cpx<T>* __restrict__ tw, int L, int nlines,
                        int ls, const int nstages, const uint64_t code, int tid, int nthr) {
  int Ns = 1;
  for (int s = 0; s < nstages; ++s) {
    const int R = (int)((code >> (4 * s)) & 15u);
    if (R == 8) fft_stage<T, 8, INV>(buf, tw, L, nlines, ls, Ns, tid, nthr);
    else if (R == 4) fft_stage<T, 4, INV>(buf, tw, L, nlines, ls, Ns, tid, nthr);
    else if (R == 2) fft_stage<T, 2, INV>(buf, tw, L, nlines, ls, Ns, tid, nthr);
    else if constexpr (!P2) {
      if (R == 7) fft_stage<T, 7, INV>(buf, tw, L, nlines, ls, Ns, tid, nthr);
      else if (R == 5) fft_stage<T, 5, INV>(buf, tw, L, nlines, ls, Ns, tid, nthr);
      else fft_stage<T, 3, INV>(buf, tw, L, nlines, ls, Ns, tid, nthr);
    }
    Ns *= R;
  }
}

inline bool is_pow2(int L) { return L > 0 && (L & (L - 1)) == 0; }

}  // namespace mmp
