// FP64 demagnetising tensor of cuboid cells and its octant spectrum.
//
// The paper (Methods, "Magnetostatic field") uses the analytic cell-cell
// result of Newell, Williams and Dunlop below a cutoff radius and an
// asymptotic result beyond it.  With r = |R| / max(d):
//   r < 3        Newell: 27-point second difference of f (diagonal) / g
//                (off-diagonal), FP64;
//   3 <= r < 40  the same cell-pair average by Gauss-Legendre quadrature of
//                the point-dipole kernel over the triangle-distributed
//                offset (each half-axis an n-point rule, n = 8 for
//                near-cubic cells, 12 otherwise), where Newell's formula
//                loses digits to cancellation;
//   r >= 40      4th-moment asymptotic expansion (second and fourth moments
//                d^2/6, d^4/15 of the triangle density), with the
//                derivatives of 1/R from the Cartesian recurrence
//                n R^2 a_k = (2n-1) sum_i x_i a_{k-e_i} - (n-1) sum_i a_{k-2e_i},
//                a_k = (-1)^|k|/k! d^k (1/R).
// Along a periodic axis (x or y) the kernel is cyclic with the grid's period
// and holds, at each cyclic offset, the sum over the images k = -R..R (the
// mean of +n/2 and -n/2 at the half period); the transform then runs over
// the cyclic offsets only.
// Each component has a definite parity per axis, so its DFT on the padded
// grid is a product of cosine/sine sums evaluated here directly in FP64
// (exact integer phase indexes into FP64 trig tables), then scaled by
// -mu0/(Px Py Pz) (and -1 for the odd-odd components, from (-i)^2).
#include "demag.h"

namespace mmp {

constexpr double kRNear = 3.0;
constexpr double kRFar = 40.0;

// ------------------------------------------------------------- Newell --
__device__ double newell_f(double x, double y, double z) {
  x = fabs(x); y = fabs(y); z = fabs(z);
  const double x2 = x * x, y2 = y * y, z2 = z * z;
  const double R = sqrt(x2 + y2 + z2);
  double out = (2.0 * x2 - y2 - z2) * R / 6.0;
  double p = 0.5 * y * (z2 - x2);
  if (p != 0.0) out += p * asinh(y / sqrt(x2 + z2));
  p = 0.5 * z * (y2 - x2);
  if (p != 0.0) out += p * asinh(z / sqrt(x2 + y2));
  p = x * y * z;
  if (p != 0.0) out -= p * atan(y * z / (x * R));
  return out;
}

__device__ double newell_g(double x, double y, double z) {
  const double sgn = (x > 0 ? 1.0 : (x < 0 ? -1.0 : 0.0)) * (y > 0 ? 1.0 : (y < 0 ? -1.0 : 0.0));
  if (sgn == 0.0) return 0.0;
  x = fabs(x); y = fabs(y); z = fabs(z);
  const double x2 = x * x, y2 = y * y, z2 = z * z;
  const double R = sqrt(x2 + y2 + z2);
  double out = -x * y * R / 3.0;
  double p = x * y * z;
  if (p != 0.0) out += p * asinh(z / sqrt(x2 + y2));
  p = y * (3.0 * z2 - y2) / 6.0;
  if (p != 0.0) out += p * asinh(x / sqrt(y2 + z2));
  p = x * (3.0 * z2 - x2) / 6.0;
  if (p != 0.0) out += p * asinh(y / sqrt(x2 + z2));
  p = z2 * z / 6.0;
  if (p != 0.0) out -= p * atan(x * y / (z * R));
  p = 0.5 * z * y2;
  if (p != 0.0) out -= p * atan(x * z / (y * R));
  p = 0.5 * z * x2;
  if (p != 0.0) out -= p * atan(y * z / (x * R));
  return sgn * out;
}

template <bool OFFDIAG>
__device__ double second_difference(double X, double Y, double Z, double dx, double dy, double dz) {
  double acc = 0.0;
  for (int a = -1; a <= 1; ++a) {
    const double wa = a == 0 ? 2.0 : -1.0;
    for (int b = -1; b <= 1; ++b) {
      const double wb = b == 0 ? 2.0 : -1.0;
      for (int c = -1; c <= 1; ++c) {
        const double wc = c == 0 ? 2.0 : -1.0;
        const double f = OFFDIAG ? newell_g(X + a * dx, Y + b * dy, Z + c * dz)
                                 : newell_f(X + a * dx, Y + b * dy, Z + c * dz);
        acc += wa * wb * wc * f;
      }
    }
  }
  return acc / (4.0 * kPi * dx * dy * dz);
}

struct TensorArgs {
  int nx, ny, nz;
  double dx, dy, dz, dmax;
  double* n6;          // [6][nz][ny][nx]
  int bx, by, bz;      // box of offsets this launch covers
  int nq;              // quadrature points per axis (2n)
  double qt[24], qw[24];
  int rx, ry;          // image repetitions along x and y (0: open axis)
};

__global__ void k_tensor_near(TensorArgs a) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long nbox = (long)a.bx * a.by * a.bz;
  if (i >= nbox) return;
  const int X = (int)(i % a.bx), Y = (int)((i / a.bx) % a.by), Z = (int)(i / ((long)a.bx * a.by));
  const double x = X * a.dx, y = Y * a.dy, z = Z * a.dz;
  const double r = sqrt(x * x + y * y + z * z) / a.dmax;
  if (r >= kRNear) return;
  const long N = (long)a.nx * a.ny * a.nz;
  const long o = ((long)Z * a.ny + Y) * a.nx + X;
  a.n6[o] = second_difference<false>(x, y, z, a.dx, a.dy, a.dz);
  a.n6[N + o] = second_difference<false>(y, x, z, a.dy, a.dx, a.dz);
  a.n6[2 * N + o] = second_difference<false>(z, y, x, a.dz, a.dy, a.dx);
  a.n6[3 * N + o] = second_difference<true>(x, y, z, a.dx, a.dy, a.dz);
  a.n6[4 * N + o] = second_difference<true>(x, z, y, a.dx, a.dz, a.dy);
  a.n6[5 * N + o] = second_difference<true>(y, z, x, a.dy, a.dz, a.dx);
}

// One block per offset of the middle regime; threads split the points.
__global__ void k_tensor_quad(TensorArgs a) {
  const long i = blockIdx.x;
  const int X = (int)(i % a.bx), Y = (int)((i / a.bx) % a.by), Z = (int)(i / ((long)a.bx * a.by));
  const double x = X * a.dx, y = Y * a.dy, z = Z * a.dz;
  const double r = sqrt(x * x + y * y + z * z) / a.dmax;
  if (r < kRNear || r >= kRFar) return;
  const int nq = a.nq;
  const int npt = nq * nq * nq;
  double acc[6] = {0, 0, 0, 0, 0, 0};
  for (int p = threadIdx.x; p < npt; p += blockDim.x) {
    const int ia = p % nq, ib = (p / nq) % nq, ic = p / (nq * nq);
    const double w = a.qw[ia] * a.qw[ib] * a.qw[ic];
    const double sx = x + a.qt[ia] * a.dx, sy = y + a.qt[ib] * a.dy, sz = z + a.qt[ic] * a.dz;
    const double s2 = sx * sx + sy * sy + sz * sz;
    const double inv5 = w / (s2 * s2 * sqrt(s2));
    acc[0] += (3.0 * sx * sx - s2) * inv5;
    acc[1] += (3.0 * sy * sy - s2) * inv5;
    acc[2] += (3.0 * sz * sz - s2) * inv5;
    acc[3] += 3.0 * sx * sy * inv5;
    acc[4] += 3.0 * sx * sz * inv5;
    acc[5] += 3.0 * sy * sz * inv5;
  }
  __shared__ double red[6][256];
  for (int c = 0; c < 6; ++c) red[c][threadIdx.x] = acc[c];
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s)
      for (int c = 0; c < 6; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const long N = (long)a.nx * a.ny * a.nz;
    const long o = ((long)Z * a.ny + Y) * a.nx + X;
    const double pref = -(a.dx * a.dy * a.dz) / (4.0 * kPi);
    for (int c = 0; c < 6; ++c) a.n6[c * N + o] = pref * red[c][0];
  }
}

// flat index of the multi-index (p, q, r), |k| = p+q+r <= 6: orders are stored
// consecutively, (p, q) ordered within an order (84 entries in all)
__device__ __forceinline__ int aidx(int p, int q, int r) {
  const int n = p + q + r;
  return n * (n + 1) * (n + 2) / 6 + p * (2 * n + 3 - p) / 2 + q;
}

// 4th-moment expansion at offset (x, y, z), |R| >= 40 max(d)
__device__ void tensor_far_at(double x, double y, double z, const TensorArgs& a, double* o6) {
  const double R2 = x * x + y * y + z * z;
  // a_k = (-1)^|k|/k! d^k (1/R) for |k| <= 6
  double A[84];
  A[aidx(0, 0, 0)] = 1.0 / sqrt(R2);
  for (int n = 1; n <= 6; ++n) {
    for (int p = 0; p <= n; ++p) {
      for (int q = 0; q <= n - p; ++q) {
        const int s = n - p - q;
        double acc = 0.0;
        if (p) acc += (2 * n - 1) * x * A[aidx(p - 1, q, s)];
        if (q) acc += (2 * n - 1) * y * A[aidx(p, q - 1, s)];
        if (s) acc += (2 * n - 1) * z * A[aidx(p, q, s - 1)];
        if (p >= 2) acc -= (n - 1) * A[aidx(p - 2, q, s)];
        if (q >= 2) acc -= (n - 1) * A[aidx(p, q - 2, s)];
        if (s >= 2) acc -= (n - 1) * A[aidx(p, q, s - 2)];
        A[aidx(p, q, s)] = acc / (n * R2);
      }
    }
  }
  const double fact[7] = {1, 1, 2, 6, 24, 120, 720};
  const double d[3] = {a.dx, a.dy, a.dz};
  const int comp_i[6] = {0, 1, 2, 0, 0, 1};
  const int comp_j[6] = {0, 1, 2, 1, 2, 2};
  const double pref = -(a.dx * a.dy * a.dz) / (4.0 * kPi);
  for (int c = 0; c < 6; ++c) {
    int base[3] = {0, 0, 0};
    base[comp_i[c]]++;
    base[comp_j[c]]++;
    auto D = [&](int e0, int e1, int e2) {
      const int p = base[0] + e0, q = base[1] + e1, s = base[2] + e2;
      const double sign = ((p + q + s) & 1) ? -1.0 : 1.0;
      return sign * fact[p] * fact[q] * fact[s] * A[aidx(p, q, s)];
    };
    double acc = D(0, 0, 0);
    acc += d[0] * d[0] / 12.0 * D(2, 0, 0) + d[1] * d[1] / 12.0 * D(0, 2, 0) +
           d[2] * d[2] / 12.0 * D(0, 0, 2);
    acc += d[0] * d[0] * d[0] * d[0] / 360.0 * D(4, 0, 0) +
           d[1] * d[1] * d[1] * d[1] / 360.0 * D(0, 4, 0) +
           d[2] * d[2] * d[2] * d[2] / 360.0 * D(0, 0, 4);
    acc += d[0] * d[0] * d[1] * d[1] / 144.0 * D(2, 2, 0) +
           d[0] * d[0] * d[2] * d[2] / 144.0 * D(2, 0, 2) +
           d[1] * d[1] * d[2] * d[2] / 144.0 * D(0, 2, 2);
    o6[c] = pref * acc;
  }
}

__global__ void k_tensor_far(TensorArgs a) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long N = (long)a.nx * a.ny * a.nz;
  if (i >= N) return;
  const int X = (int)(i % a.nx), Y = (int)((i / a.nx) % a.ny), Z = (int)(i / ((long)a.nx * a.ny));
  const double x = X * a.dx, y = Y * a.dy, z = Z * a.dz;
  const double r = sqrt(x * x + y * y + z * z) / a.dmax;
  if (r < kRFar) return;
  double o6[6];
  tensor_far_at(x, y, z, a, o6);
  for (int c = 0; c < 6; ++c) a.n6[c * N + i] = o6[c];
}

// The tensor at any offset, regime by distance; the middle regime's
// quadrature runs in the calling thread.
__device__ void tensor_at(double x, double y, double z, const TensorArgs& a, double* o6) {
  const double r = sqrt(x * x + y * y + z * z) / a.dmax;
  if (r < kRNear) {
    o6[0] = second_difference<false>(x, y, z, a.dx, a.dy, a.dz);
    o6[1] = second_difference<false>(y, x, z, a.dy, a.dx, a.dz);
    o6[2] = second_difference<false>(z, y, x, a.dz, a.dy, a.dx);
    o6[3] = second_difference<true>(x, y, z, a.dx, a.dy, a.dz);
    o6[4] = second_difference<true>(x, z, y, a.dx, a.dz, a.dy);
    o6[5] = second_difference<true>(y, z, x, a.dy, a.dz, a.dx);
  } else if (r < kRFar) {
    double acc[6] = {0, 0, 0, 0, 0, 0};
    const int nq = a.nq;
    for (int ic = 0; ic < nq; ++ic)
      for (int ib = 0; ib < nq; ++ib)
        for (int ia = 0; ia < nq; ++ia) {
          const double w = a.qw[ia] * a.qw[ib] * a.qw[ic];
          const double sx = x + a.qt[ia] * a.dx, sy = y + a.qt[ib] * a.dy,
                       sz = z + a.qt[ic] * a.dz;
          const double s2 = sx * sx + sy * sy + sz * sz;
          const double inv5 = w / (s2 * s2 * sqrt(s2));
          acc[0] += (3.0 * sx * sx - s2) * inv5;
          acc[1] += (3.0 * sy * sy - s2) * inv5;
          acc[2] += (3.0 * sz * sz - s2) * inv5;
          acc[3] += 3.0 * sx * sy * inv5;
          acc[4] += 3.0 * sx * sz * inv5;
          acc[5] += 3.0 * sy * sz * inv5;
        }
    const double pref = -(a.dx * a.dy * a.dz) / (4.0 * kPi);
    for (int c = 0; c < 6; ++c) o6[c] = pref * acc[c];
  } else {
    tensor_far_at(x, y, z, a, o6);
  }
}

// Periodic axes: the tensor at offsets 0 <= X <= nx/2 (and/or Y) summed over
// the images X + k nx, k = -rx..rx; at the half period (X = nx/2, nx even)
// the offsets +X and -X are one cyclic index holding their mean, so a
// component odd along that axis is zero there.  Open axes cover 0 <= X < n.
__global__ void k_tensor_images(TensorArgs a) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long nbox = (long)a.bx * a.by * a.bz;
  if (i >= nbox) return;
  const int X = (int)(i % a.bx), Y = (int)((i / a.bx) % a.by), Z = (int)(i / ((long)a.bx * a.by));
  double sum[6] = {0, 0, 0, 0, 0, 0};
  for (int ky = -a.ry; ky <= a.ry; ++ky)
    for (int kx = -a.rx; kx <= a.rx; ++kx) {
      double o6[6];
      tensor_at((X + (double)kx * a.nx) * a.dx, (Y + (double)ky * a.ny) * a.dy, Z * a.dz, a, o6);
      for (int c = 0; c < 6; ++c) sum[c] += o6[c];
    }
  const bool hx = a.rx > 0 && 2 * X == a.nx, hy = a.ry > 0 && 2 * Y == a.ny;
  const int oddx[6] = {0, 0, 0, 1, 1, 0}, oddy[6] = {0, 0, 0, 1, 0, 1};
  const long N = (long)a.nx * a.ny * a.nz;
  const long o = ((long)Z * a.ny + Y) * a.nx + X;
  for (int c = 0; c < 6; ++c)
    a.n6[c * N + o] = ((hx && oddx[c]) || (hy && oddy[c])) ? 0.0 : sum[c];
}

// --------------------------------------------------- trig transforms ----
__global__ void k_trig_table(double* cs, double* sn, int P) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= P) return;
  double s, c;
  sincospi(2.0 * (double)j / (double)P, &s, &c);
  cs[j] = c;
  sn[j] = s;
}

// parity per component (xx, yy, zz, xy, xz, yz): odd in x / y / z
__constant__ int kOddX[6] = {0, 0, 0, 1, 1, 0};
__constant__ int kOddY[6] = {0, 0, 0, 1, 0, 1};
__constant__ int kOddZ[6] = {0, 0, 0, 0, 1, 1};

// weight of offset X in a cosine/sine sum over X >= 0: offsets +X and -X
// both, except X = 0 and, on a periodic axis, the half period X = n/2
__device__ __forceinline__ double offset_weight(int X, int n, int per) {
  return (X == 0 || (per && 2 * X == n)) ? 1.0 : 2.0;
}

// F1[c][Z][Y][kx] = sum_X w_X N[c][Z][Y][X] trig(kx X); a periodic axis
// sums 0 <= X <= nx/2 (the cyclic offsets), an open one 0 <= X < nx
__global__ void k_trig_x(const double* n6, double* f1, const double* cs, const double* sn,
                         int nx, int ny, int nz, int Px, int Hx, int per) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long tot = 6L * nz * ny * Hx;
  if (i >= tot) return;
  const int kx = (int)(i % Hx);
  const long row = i / Hx;  // (c, Z, Y)
  const int c = (int)(row / ((long)nz * ny));
  const double* tab = kOddX[c] ? sn : cs;
  const double* in = n6 + row * nx;
  const int xe = per ? nx / 2 + 1 : nx;
  double acc = 0.0;
  for (int X = 0; X < xe; ++X)
    acc += offset_weight(X, nx, per) * in[X] * tab[(int)(((long)kx * X) % Px)];
  f1[i] = acc;
}

// F2[c][Z][ky][kx] = sum_Y w_Y F1[c][Z][Y][kx] trig(ky Y), ky <= Py/2
__global__ void k_trig_y(const double* f1, double* f2, const double* cs, const double* sn,
                         int ny, int nz, int Py, int Hx, int Hy, int per) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long tot = 6L * nz * Hy * Hx;
  if (i >= tot) return;
  const int kx = (int)(i % Hx);
  const int ky = (int)((i / Hx) % Hy);
  const long cz = i / ((long)Hx * Hy);  // (c, Z)
  const int c = (int)(cz / nz);
  const double* tab = kOddY[c] ? sn : cs;
  const double* in = f1 + cz * ny * Hx + kx;
  const int ye = per ? ny / 2 + 1 : ny;
  double acc = 0.0;
  for (int Y = 0; Y < ye; ++Y)
    acc += offset_weight(Y, ny, per) * in[(long)Y * Hx] * tab[(int)(((long)ky * Y) % Py)];
  f2[i] = acc;
}

// K[c][kz][kx][ky] = scale_c sum_Z w_Z F2[c][Z][ky][kx] trig(kz Z), kz <= Pz/2
template <typename T>
__global__ void k_trig_z(const double* f2, T* kout, double* k64, const double* cs,
                         const double* sn, int nz, int Pz, int Hx, int Hy, int Hz, double scale) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long tot = 6L * Hz * Hy * Hx;
  if (i >= tot) return;
  const int kx = (int)(i % Hx);
  const int ky = (int)((i / Hx) % Hy);
  const int kz = (int)((i / ((long)Hx * Hy)) % Hz);
  const int c = (int)(i / ((long)Hx * Hy * Hz));
  const double* tab = kOddZ[c] ? sn : cs;
  const double* in = f2 + (long)c * nz * Hy * Hx + (long)ky * Hx + kx;
  double acc = 0.0;
  for (int Z = 0; Z < nz; ++Z) {
    const double w = Z == 0 ? 1.0 : 2.0;
    acc += w * in[(long)Z * Hy * Hx] * tab[(int)(((long)kz * Z) % Pz)];
  }
  const double sc = c >= 3 ? -scale : scale;
  const long o = (((long)c * Hz + kz) * Hx + kx) * Hy + ky;
  kout[o] = (T)(sc * acc);
  if (k64) k64[o] = sc * acc;
}

// ---------------------------------------------------------- host side --
static void gauss_legendre(int n, double* x, double* w) {
  for (int i = 0; i < n; ++i) {
    double z = std::cos(kPi * (i + 0.75) / (n + 0.5));
    double pp = 0.0;
    for (int it = 0; it < 100; ++it) {
      double p1 = 1.0, p2 = 0.0;
      for (int j = 1; j <= n; ++j) {
        const double p3 = p2;
        p2 = p1;
        p1 = ((2.0 * j - 1.0) * z * p2 - (j - 1.0) * p3) / j;
      }
      pp = n * (z * p1 - p2) / (z * z - 1.0);
      const double z1 = z;
      z = z1 - p1 / pp;
      if (std::fabs(z - z1) < 1e-16) {
        // one more evaluation of the derivative at the converged root
        p1 = 1.0; p2 = 0.0;
        for (int j = 1; j <= n; ++j) {
          const double p3 = p2;
          p2 = p1;
          p1 = ((2.0 * j - 1.0) * z * p2 - (j - 1.0) * p3) / j;
        }
        pp = n * (z * p1 - p2) / (z * z - 1.0);
        break;
      }
    }
    x[i] = z;
    w[i] = 2.0 / ((1.0 - z * z) * pp * pp);
  }
}

// nodes on [-1, 1] for the density (1 - |t|), 2n of them
static void triangle_rule(int n, double* t, double* w) {
  double x[12], gw[12];
  gauss_legendre(n, x, gw);
  for (int i = 0; i < n; ++i) {
    const double tp = 0.5 * (x[i] + 1.0);
    const double wp = 0.5 * gw[i] * (1.0 - tp);
    t[n + i] = tp;
    w[n + i] = wp;
    t[n - 1 - i] = -tp;
    w[n - 1 - i] = wp;
  }
}

static int fill_tensor(int nx, int ny, int nz, double dx, double dy, double dz, double* n6,
                       hipStream_t st) {
  TensorArgs a{};
  a.nx = nx; a.ny = ny; a.nz = nz;
  a.dx = dx; a.dy = dy; a.dz = dz;
  a.dmax = std::fmax(dx, std::fmax(dy, dz));
  const double dmin = std::fmin(dx, std::fmin(dy, dz));
  const int n = (a.dmax / dmin <= 1.25) ? 8 : 12;
  a.nq = 2 * n;
  triangle_rule(n, a.qt, a.qw);
  a.n6 = n6;
  auto box = [&](double rcut, int nn, double d) {
    const int b = (int)std::ceil(rcut * a.dmax / d) + 1;
    return b < nn ? b : nn;
  };
  // near
  a.bx = box(kRNear, nx, dx); a.by = box(kRNear, ny, dy); a.bz = box(kRNear, nz, dz);
  long nb = (long)a.bx * a.by * a.bz;
  hipLaunchKernelGGL(k_tensor_near, dim3((unsigned)((nb + 127) / 128)), dim3(128), 0, st, a);
  // middle
  a.bx = box(kRFar, nx, dx); a.by = box(kRFar, ny, dy); a.bz = box(kRFar, nz, dz);
  nb = (long)a.bx * a.by * a.bz;
  hipLaunchKernelGGL(k_tensor_quad, dim3((unsigned)nb), dim3(256), 0, st, a);
  // far
  const long N = (long)nx * ny * nz;
  hipLaunchKernelGGL(k_tensor_far, dim3((unsigned)((N + 127) / 128)), dim3(128), 0, st, a);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int demag_tensor_only(int nx, int ny, int nz, double dx, double dy, double dz, double* n6,
                      hipStream_t st) {
  return fill_tensor(nx, ny, nz, dx, dy, dz, n6, st);
}

// The image-summed tensor of a grid periodic along x and/or y.
static int fill_tensor_images(int nx, int ny, int nz, double dx, double dy, double dz, int rx,
                              int ry, double* n6, hipStream_t st) {
  TensorArgs a{};
  a.nx = nx; a.ny = ny; a.nz = nz;
  a.dx = dx; a.dy = dy; a.dz = dz;
  a.dmax = std::fmax(dx, std::fmax(dy, dz));
  const double dmin = std::fmin(dx, std::fmin(dy, dz));
  const int n = (a.dmax / dmin <= 1.25) ? 8 : 12;
  a.nq = 2 * n;
  triangle_rule(n, a.qt, a.qw);
  a.n6 = n6;
  a.rx = rx; a.ry = ry;
  a.bx = rx > 0 ? nx / 2 + 1 : nx;
  a.by = ry > 0 ? ny / 2 + 1 : ny;
  a.bz = nz;
  const long nb = (long)a.bx * a.by * a.bz;
  hipLaunchKernelGGL(k_tensor_images, dim3((unsigned)((nb + 63) / 64)), dim3(64), 0, st, a);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// Tensor between the cells of a layer at height z_t (centre, layer 0 of the
// grid centred at 0) and the grid's cells: k6[c][z][Y + ny - 1][X + nx - 1]
// = N(X dx, Y dy, z_t - z dz) for |X| < nx, |Y| < ny.
__global__ void k_tensor_layer(TensorArgs a, double zt, double* k6) {
  const int wx = 2 * a.nx - 1, wy = 2 * a.ny - 1;
  const long tot = (long)wx * wy * a.nz;
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= tot) return;
  const int ix = (int)(i % wx), iy = (int)((i / wx) % wy), z = (int)(i / ((long)wx * wy));
  double o6[6];
  tensor_at((ix - (a.nx - 1)) * a.dx, (iy - (a.ny - 1)) * a.dy, zt - z * a.dz, a, o6);
  for (int c = 0; c < 6; ++c) k6[(long)c * tot + i] = o6[c];
}

int stray_kernel_build(int nx, int ny, int nz, double dx, double dy, double dz, double zt,
                       double* k6, hipStream_t st) {
  TensorArgs a{};
  a.nx = nx; a.ny = ny; a.nz = nz;
  a.dx = dx; a.dy = dy; a.dz = dz;
  a.dmax = std::fmax(dx, std::fmax(dy, dz));
  const double dmin = std::fmin(dx, std::fmin(dy, dz));
  const int n = (a.dmax / dmin <= 1.25) ? 8 : 12;
  a.nq = 2 * n;
  triangle_rule(n, a.qt, a.qw);
  const long tot = (long)(2 * nx - 1) * (2 * ny - 1) * nz;
  hipLaunchKernelGGL(k_tensor_layer, dim3((unsigned)((tot + 63) / 64)), dim3(64), 0, st, a, zt,
                     k6);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <typename T>
int demag_kernel_build(const DemagPlan& p, double dx, double dy, double dz, double* n6, T* kout,
                       hipStream_t st) {
  if (p.rep[0] > 0 || p.rep[1] > 0) {
    if (fill_tensor_images(p.nx, p.ny, p.nz, dx, dy, dz, p.rep[0], p.rep[1], n6, st)) return -1;
  } else if (fill_tensor(p.nx, p.ny, p.nz, dx, dy, dz, n6, st)) {
    return -1;
  }
  DeviceLock lk(device_mutex());
  double *f1 = nullptr, *f2 = nullptr, *tabs = nullptr;
  const size_t n1 = (size_t)6 * p.nz * p.ny * p.Hx;
  const size_t n2 = (size_t)6 * p.nz * p.Hy * p.Hx;
  const int Pm = p.Px + p.Py + p.Pz;
  if (hipMalloc(&f1, n1 * sizeof(double)) != hipSuccess) return -2;
  if (hipMalloc(&f2, n2 * sizeof(double)) != hipSuccess) { (void)hipFree(f1); return -2; }
  if (hipMalloc(&tabs, (size_t)2 * Pm * sizeof(double)) != hipSuccess) {
    (void)hipFree(f1); (void)hipFree(f2); return -2;
  }
  double* cx = tabs;            double* sx = cx + p.Px;
  double* cy = sx + p.Px;       double* sy = cy + p.Py;
  double* cz = sy + p.Py;       double* sz = cz + p.Pz;
  hipLaunchKernelGGL(k_trig_table, dim3((p.Px + 255) / 256), dim3(256), 0, st, cx, sx, p.Px);
  hipLaunchKernelGGL(k_trig_table, dim3((p.Py + 255) / 256), dim3(256), 0, st, cy, sy, p.Py);
  hipLaunchKernelGGL(k_trig_table, dim3((p.Pz + 255) / 256), dim3(256), 0, st, cz, sz, p.Pz);
  hipLaunchKernelGGL(k_trig_x, dim3((unsigned)((n1 + 255) / 256)), dim3(256), 0, st, n6, f1, cx,
                     sx, p.nx, p.ny, p.nz, p.Px, p.Hx, p.rep[0] > 0 ? 1 : 0);
  hipLaunchKernelGGL(k_trig_y, dim3((unsigned)((n2 + 255) / 256)), dim3(256), 0, st, f1, f2, cy,
                     sy, p.ny, p.nz, p.Py, p.Hx, p.Hy, p.rep[1] > 0 ? 1 : 0);
  const double scale = -kMu0 / ((double)p.Px * p.Py * p.Pz);
  hipLaunchKernelGGL((k_trig_z<T>), dim3((unsigned)((p.k_elems + 255) / 256)), dim3(256), 0, st,
                     f2, kout, (double*)nullptr, cz, sz, p.nz, p.Pz, p.Hx, p.Hy, p.Hz, scale);
  const hipError_t e = hipStreamSynchronize(st);
  (void)hipFree(f1);
  (void)hipFree(f2);
  (void)hipFree(tabs);
  return e == hipSuccess ? 0 : -1;
}

template int demag_kernel_build<float>(const DemagPlan&, double, double, double, double*, float*,
                                       hipStream_t);
template int demag_kernel_build<double>(const DemagPlan&, double, double, double, double*,
                                        double*, hipStream_t);

}  // namespace mmp
