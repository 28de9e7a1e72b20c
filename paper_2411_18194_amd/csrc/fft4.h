// Register-resident FFTs and the four-step line transform (power-of-two
// lengths) for gfx950.
//
// reg_fft<N>: an N-point FFT (N <= 64) held entirely in one thread's
// registers, Stockham autosort with radix 8/4/2 butterflies; every index and
// twiddle is a compile-time constant, so the data movement is register
// renaming and the twiddles are literals.
//
// Four-step line transform of length L = L1*L2 (L1 = L2 or 2*L2): with
// n = L2*n1 + n2 and k = k1 + L1*k2,
//   X[k1 + L1 k2] = sum_n2 w_L^(n2 k1) w_L2^(n2 k2) sum_n1 x[L2 n1 + n2] w_L1^(n1 k1).
// Thread t (one of L2 per line) loads x[L2 n1 + t] (coalesced across t),
// does the L1-point transform in registers, multiplies by w_L^(t k1) (table
// laid out [k1][t] so the loads are coalesced), and writes row k1 of an LDS
// transpose whose columns are XOR-swizzled by k1 (conflict-free both ways);
// after one barrier it reads back L2-point columns, transforms them in
// registers and holds X[k1 + L1 k2] for k1 = t + L2 i.
#pragma once

#include "common.h"

namespace mmp {

// cos/sin(2 pi j / 64), j = 0..63
struct Root64 {
  static constexpr double c[64] = {
    1.00000000000000000000e+00, 9.95184726672196928732e-01, 9.80785280403230430579e-01, 9.56940335732208824382e-01,
    9.23879532511286738483e-01, 8.81921264348355049556e-01, 8.31469612302545235671e-01, 7.73010453362736993377e-01,
    7.07106781186547572737e-01, 6.34393284163645487794e-01, 5.55570233019602288671e-01, 4.71396736825997808573e-01,
    3.82683432365089837290e-01, 2.90284677254462331053e-01, 1.95090322016128331351e-01, 9.80171403295607701622e-02,
    6.12323399573676603587e-17, -9.80171403295606452621e-02, -1.95090322016128192573e-01, -2.90284677254462164520e-01,
    -3.82683432365089726268e-01, -4.71396736825997697551e-01, -5.55570233019601955604e-01, -6.34393284163645376772e-01,
    -7.07106781186547461715e-01, -7.73010453362736993377e-01, -8.31469612302545346694e-01, -8.81921264348354938534e-01,
    -9.23879532511286738483e-01, -9.56940335732208824382e-01, -9.80785280403230430579e-01, -9.95184726672196817709e-01,
    -1.00000000000000000000e+00, -9.95184726672196928732e-01, -9.80785280403230430579e-01, -9.56940335732208935404e-01,
    -9.23879532511286849505e-01, -8.81921264348355049556e-01, -8.31469612302545457716e-01, -7.73010453362737104399e-01,
    -7.07106781186547683760e-01, -6.34393284163645931883e-01, -5.55570233019602177649e-01, -4.71396736825997864084e-01,
    -3.82683432365090336891e-01, -2.90284677254462442075e-01, -1.95090322016128664417e-01, -9.80171403295604509731e-02,
    -1.83697019872102968750e-16, 9.80171403295600901506e-02, 1.95090322016128303595e-01, 2.90284677254462053497e-01,
    3.82683432365090003824e-01, 4.71396736825997586529e-01, 5.55570233019601844582e-01, 6.34393284163645598817e-01,
    7.07106781186547350693e-01, 7.73010453362736660310e-01, 8.31469612302545235671e-01, 8.81921264348354827511e-01,
    9.23879532511286516439e-01, 9.56940335732208824382e-01, 9.80785280403230319557e-01, 9.95184726672196928732e-01,
  };
  static constexpr double s[64] = {
    0.00000000000000000000e+00, 9.80171403295606036288e-02, 1.95090322016128248084e-01, 2.90284677254462331053e-01,
    3.82683432365089781779e-01, 4.71396736825997642040e-01, 5.55570233019602177649e-01, 6.34393284163645487794e-01,
    7.07106781186547461715e-01, 7.73010453362736993377e-01, 8.31469612302545235671e-01, 8.81921264348354938534e-01,
    9.23879532511286738483e-01, 9.56940335732208935404e-01, 9.80785280403230430579e-01, 9.95184726672196817709e-01,
    1.00000000000000000000e+00, 9.95184726672196928732e-01, 9.80785280403230430579e-01, 9.56940335732208935404e-01,
    9.23879532511286738483e-01, 8.81921264348355049556e-01, 8.31469612302545457716e-01, 7.73010453362737104399e-01,
    7.07106781186547572737e-01, 6.34393284163645487794e-01, 5.55570233019602177649e-01, 4.71396736825997864084e-01,
    3.82683432365089892802e-01, 2.90284677254462386564e-01, 1.95090322016128608906e-01, 9.80171403295608256734e-02,
    1.22464679914735320717e-16, -9.80171403295605897510e-02, -1.95090322016128359106e-01, -2.90284677254462109008e-01,
    -3.82683432365089670757e-01, -4.71396736825997642040e-01, -5.55570233019601955604e-01, -6.34393284163645265750e-01,
    -7.07106781186547461715e-01, -7.73010453362736660310e-01, -8.31469612302545235671e-01, -8.81921264348354938534e-01,
    -9.23879532511286516439e-01, -9.56940335732208824382e-01, -9.80785280403230319557e-01, -9.95184726672196928732e-01,
    -1.00000000000000000000e+00, -9.95184726672196928732e-01, -9.80785280403230430579e-01, -9.56940335732208935404e-01,
    -9.23879532511286627461e-01, -8.81921264348355049556e-01, -8.31469612302545457716e-01, -7.73010453362736882355e-01,
    -7.07106781186547683760e-01, -6.34393284163645931883e-01, -5.55570233019602177649e-01, -4.71396736825997919595e-01,
    -3.82683432365090392402e-01, -2.90284677254462497586e-01, -1.95090322016128719929e-01, -9.80171403295605064843e-02,
  };
};

// exp(sign 2 pi i e / M) for compile-time e, M (M divides 64 or M <= 64)
template <typename T, int E, int M, bool INV>
__device__ __forceinline__ cpx<T> root() {
  constexpr int j = ((E % M) * (64 / M)) % 64;
  return cmk<T>(T(Root64::c[j]), INV ? T(Root64::s[j]) : T(-Root64::s[j]));
}

template <typename T, int R, bool INV>
__device__ __forceinline__ void bfly(cpx<T>* v);

template <typename T, int R, bool INV>
__device__ __forceinline__ void bfly(cpx<T>* v) {
  using V = cpx<T>;
  if constexpr (R == 2) {
    V a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  } else if constexpr (R == 4) {
    V s02 = cadd(v[0], v[2]), d02 = csub(v[0], v[2]);
    V s13 = cadd(v[1], v[3]), d13 = csub(v[1], v[3]);
    V jd = INV ? cmk<T>(-d13.y, d13.x) : cmk<T>(d13.y, -d13.x);
    v[0] = cadd(s02, s13);
    v[2] = csub(s02, s13);
    v[1] = cadd(d02, jd);
    v[3] = csub(d02, jd);
  } else {
    static_assert(R == 8, "radix");
    const T h = T(0.70710678118654752440);
    V a[4], b[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      a[r] = cadd(v[r], v[r + 4]);
      b[r] = csub(v[r], v[r + 4]);
    }
    if (!INV) {
      b[1] = cmk<T>(h * (b[1].x + b[1].y), h * (b[1].y - b[1].x));
      b[2] = cmk<T>(b[2].y, -b[2].x);
      b[3] = cmk<T>(h * (b[3].y - b[3].x), -h * (b[3].x + b[3].y));
    } else {
      b[1] = cmk<T>(h * (b[1].x - b[1].y), h * (b[1].y + b[1].x));
      b[2] = cmk<T>(-b[2].y, b[2].x);
      b[3] = cmk<T>(-h * (b[3].x + b[3].y), h * (b[3].x - b[3].y));
    }
    bfly<T, 4, INV>(a);
    bfly<T, 4, INV>(b);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      v[2 * k] = a[k];
      v[2 * k + 1] = b[k];
    }
  }
}

// bit reversal of k over log2(N) bits (compile-time)
template <int N>
__host__ __device__ constexpr int bitrev(int k) {
  int r = 0;
  for (int n = N; n > 1; n >>= 1) {
    r = (r << 1) | (k & 1);
    k >>= 1;
  }
  return r;
}

// multiply by exp(-/+ 2 pi i e / M) with the trivial angles done exactly
template <typename T, int E, int M, bool INV>
__device__ __forceinline__ cpx<T> twiddle_c(cpx<T> x) {
  constexpr int jj = ((E % M) * (64 / M)) % 64;  // angle in units of 2 pi/64
  if constexpr (jj == 0) {
    return x;
  } else if constexpr (jj == 16) {  // -/+ i
    return INV ? cmk<T>(-x.y, x.x) : cmk<T>(x.y, -x.x);
  } else if constexpr (jj == 32) {
    return cmk<T>(-x.x, -x.y);
  } else if constexpr (jj == 48) {
    return INV ? cmk<T>(x.y, -x.x) : cmk<T>(-x.y, x.x);
  } else {
    const cpx<T> w = cmk<T>(T(Root64::c[jj]), INV ? T(Root64::s[jj]) : T(-Root64::s[jj]));
    return cmul(x, w);
  }
}

// one radix-2 decimation-in-frequency level with half-span H on blocks of 2H
template <typename T, int N, int H, bool INV, int I>
__device__ __forceinline__ void dif_level_unrolled(cpx<T>* v) {
  if constexpr (I < N / 2) {
    constexpr int blk = I / H, j = I % H;
    constexpr int i0 = blk * 2 * H + j, i1 = i0 + H;
    const cpx<T> a = v[i0], b = v[i1];
    v[i0] = cadd(a, b);
    v[i1] = twiddle_c<T, j, 2 * H, INV>(csub(a, b));
    dif_level_unrolled<T, N, H, INV, I + 1>(v);
  }
}

template <typename T, int N, int H, bool INV>
__device__ __forceinline__ void dif_levels(cpx<T>* v) {
  if constexpr (H >= 1) {
    dif_level_unrolled<T, N, H, INV, 0>(v);
    dif_levels<T, N, H / 2, INV>(v);
  }
}

template <typename T, int N, bool INV, int I>
__device__ __forceinline__ void dif_first_halfzero(cpx<T>* v) {
  if constexpr (I < N / 2) {
    v[I + N / 2] = twiddle_c<T, I, N, INV>(v[I]);
    dif_first_halfzero<T, N, INV, I + 1>(v);
  }
}

// As reg_fft, for an input whose upper half v[N/2 .. N) is zero (it is not
// read): a zero-padded line whose pad is at least as long as its data.
template <typename T, int N, bool INV>
__device__ __forceinline__ void reg_fft_hz(cpx<T>* v) {
  if constexpr (N > 1) {
    dif_first_halfzero<T, N, INV, 0>(v);
    dif_levels<T, N, N / 4, INV>(v);
  }
}

// In-register N-point FFT in place (N power of two <= 64): on return the
// transform value X[k] sits in v[bitrev<N>(k)].  Only a couple of complex
// temporaries are live besides v.
template <typename T, int N, bool INV>
__device__ __forceinline__ void reg_fft(cpx<T>* v) {
  if constexpr (N > 1) dif_levels<T, N, N / 2, INV>(v);
}

// Four-step geometry for L = 2^p: L1 = L2 or 2 L2.
template <int L>
struct Split {
  static constexpr int lg = (L <= 1) ? 0 : 1 + Split<L / 2>::lg;
  static constexpr int L2 = 1 << (lg / 2);
  static constexpr int L1 = L / L2;
};
template <>
struct Split<1> {
  static constexpr int lg = 0;
  static constexpr int L2 = 1;
  static constexpr int L1 = 1;
};

}  // namespace mmp
