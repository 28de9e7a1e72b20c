// Elastodynamics on the magnet's grid (paper, Methods "Elasticity" and
// "Magnetoelasticity"): rho d2u/dt2 = div sigma + sum_s f_mel^(s) - eta v,
// integrated as (u, v) inside the same Runge-Kutta stages as m.
//
// Derivatives: 4th-order central (-f2 + 8 f1 - 8 f-1 + f-2)/(12 d) in the
// bulk, 2nd-order central one cell in from a face, 1st-order one-sided on a
// face cell (the paper uses lower-order schemes near and at boundaries); an
// axis with one cell has no derivative.  Strain is the symmetrised
// gradient of u, stress the cubic law plus the viscous stress beta C : eps(v)
// of stiffness-proportional Rayleigh damping; on each face of an axis with more
// than one cell the face cell's stress row along that axis is the traction
// (zero, i.e. traction-free), and the drive sigma_xz = A sin(w t) on x = 0
// is applied last.  The force is the divergence of that stress plus the
// magnetoelastic force of Eq. 8 per sublattice.
#include "elastic.h"

namespace mmp {

// The five points are loaded unconditionally from offsets clamped to the
// axis (so all loads of a cell go out together), then the scheme of this
// position is applied.
template <typename T>
__device__ __forceinline__ T d1(const T* __restrict__ f, long idx, int i, int n, long s, T h) {
  const long om2 = (long)(max(i - 2, 0) - i) * s, om1 = (long)(max(i - 1, 0) - i) * s;
  const long op1 = (long)(min(i + 1, n - 1) - i) * s, op2 = (long)(min(i + 2, n - 1) - i) * s;
  const T fm2 = f[idx + om2], fm1 = f[idx + om1], f0 = f[idx], fp1 = f[idx + op1],
          fp2 = f[idx + op2];
  // every candidate is formed (selects, not branches, so no load is sunk
  // into a branch)
  const T r_lo = (fp1 - f0) / h, r_hi = (f0 - fm1) / h;
  const T r_c2 = (fp1 - fm1) / (T(2) * h);
  const T r_c4 = (-fp2 + T(8) * fp1 - T(8) * fm1 + fm2) / (T(12) * h);
  const T r = (i == 1 || i == n - 2) ? r_c2 : r_c4;
  return n == 1 ? T(0) : (i == 0 ? r_lo : (i == n - 1 ? r_hi : r));
}

template <typename T>
__device__ __forceinline__ const T* u_in(const Table<T>* t, int s) {
  if (s == 0 || s == 1) return t->un;
  if (s == t->ns) return t->unew;
  return (s & 1) ? t->usb : t->usa;
}
template <typename T>
__device__ __forceinline__ const T* v_in(const Table<T>* t, int s) {
  if (s == 0 || s == 1) return t->vn;
  if (s == t->ns) return t->vnew;
  return (s & 1) ? t->vsb : t->vsa;
}
template <typename T>
__device__ __forceinline__ T* u_out(const Table<T>* t, int s) {
  const int n = s + 1;
  if (n == t->ns) return t->unew;
  return (n & 1) ? t->usb : t->usa;
}
template <typename T>
__device__ __forceinline__ T* v_out(const Table<T>* t, int s) {
  const int n = s + 1;
  if (n == t->ns) return t->vnew;
  return (n & 1) ? t->vsb : t->vsa;
}

template <typename T>
__global__ void k_strain(ElasticArgs<T> a) {
  if (ctrl_stopped(a.ctrl)) return;
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.N) return;
  const int x = (int)(i % a.nx), y = (int)((i / a.nx) % a.ny), z = (int)(i / ((long)a.nx * a.ny));
  const T* u = u_in(a.tbl, a.stage);
  const long N = a.N, sx = 1, sy = a.nx, sz = (long)a.nx * a.ny;
  T g[3][3];  // g[i][j] = d_i u_j
  for (int j = 0; j < 3; ++j) {
    const T* uj = u + j * N;
    g[0][j] = d1(uj, i, x, a.nx, sx, a.dx);
    g[1][j] = d1(uj, i, y, a.ny, sy, a.dy);
    g[2][j] = d1(uj, i, z, a.nz, sz, a.dz);
  }
  a.eps[i] = g[0][0];
  a.eps[N + i] = g[1][1];
  a.eps[2 * N + i] = g[2][2];
  a.eps[3 * N + i] = T(0.5) * (g[0][1] + g[1][0]);
  a.eps[4 * N + i] = T(0.5) * (g[0][2] + g[2][0]);
  a.eps[5 * N + i] = T(0.5) * (g[1][2] + g[2][1]);
  if (a.beta != T(0)) {
    // strain rate: the same operator on the velocity
    const T* v = v_in(a.tbl, a.stage);
    for (int j = 0; j < 3; ++j) {
      const T* vj = v + j * N;
      g[0][j] = d1(vj, i, x, a.nx, sx, a.dx);
      g[1][j] = d1(vj, i, y, a.ny, sy, a.dy);
      g[2][j] = d1(vj, i, z, a.nz, sz, a.dz);
    }
    a.epsv[i] = g[0][0];
    a.epsv[N + i] = g[1][1];
    a.epsv[2 * N + i] = g[2][2];
    a.epsv[3 * N + i] = T(0.5) * (g[0][1] + g[1][0]);
    a.epsv[4 * N + i] = T(0.5) * (g[0][2] + g[2][0]);
    a.epsv[5 * N + i] = T(0.5) * (g[1][2] + g[2][1]);
  }
}

// Voigt slot of (row, col)
__device__ __forceinline__ int voigt(int r, int c) {
  if (r == c) return r;
  const int s = r + c;  // 1: xy, 2: xz, 3: yz
  return s == 1 ? 3 : (s == 2 ? 4 : 5);
}

template <typename T>
__global__ void k_stress(ElasticArgs<T> a, int eval) {
  if (ctrl_stopped(a.ctrl)) return;
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  double e_el = 0.0;
  if (i < a.N) {
    const long N = a.N;
    const int x = (int)(i % a.nx), y = (int)((i / a.nx) % a.ny), z = (int)(i / ((long)a.nx * a.ny));
    T e[6];
    for (int c = 0; c < 6; ++c) e[c] = a.eps[c * N + i];
    T s[6];
    s[0] = a.C11 * e[0] + a.C12 * (e[1] + e[2]);
    s[1] = a.C11 * e[1] + a.C12 * (e[0] + e[2]);
    s[2] = a.C11 * e[2] + a.C12 * (e[0] + e[1]);
    s[3] = T(2) * a.C44 * e[3];
    s[4] = T(2) * a.C44 * e[4];
    s[5] = T(2) * a.C44 * e[5];
    if (eval) {
      const T* v = v_in(a.tbl, 1);
      double w = 0.0;
      for (int c = 0; c < 3; ++c) w += (double)s[c] * e[c];
      for (int c = 3; c < 6; ++c) w += 2.0 * (double)s[c] * e[c];
      double kv = 0.0;
      for (int c = 0; c < 3; ++c) kv += (double)v[c * N + i] * v[c * N + i];
      e_el = (0.5 * w + 0.5 * a.rho * kv) * a.V;
    }
    if (a.beta != T(0)) {
      // viscous stress beta C : eps(v) (stiffness-proportional Rayleigh damping)
      T r[6];
      for (int c = 0; c < 6; ++c) r[c] = a.epsv[c * N + i];
      s[0] += a.beta * (a.C11 * r[0] + a.C12 * (r[1] + r[2]));
      s[1] += a.beta * (a.C11 * r[1] + a.C12 * (r[0] + r[2]));
      s[2] += a.beta * (a.C11 * r[2] + a.C12 * (r[0] + r[1]));
      s[3] += a.beta * (T(2) * a.C44 * r[3]);
      s[4] += a.beta * (T(2) * a.C44 * r[4]);
      s[5] += a.beta * (T(2) * a.C44 * r[5]);
    }
    const int pos[3] = {x, y, z};
    const int n[3] = {a.nx, a.ny, a.nz};
    for (int k = 0; k < 3; ++k) {
      if (n[k] < 2) continue;
      if (pos[k] == 0 || pos[k] == n[k] - 1)
        for (int j = 0; j < 3; ++j) s[voigt(k, j)] = T(0);
    }
    if (a.trac_amp != 0.0 && a.nx >= 2 && x == 0) {
      const double ts = a.ctrl ? a.ctrl->t + (a.stage > 0 ? RK::t[a.tbl->rk].c[a.stage - 1] * a.ctrl->h : 0.0)
                               : 0.0;
      s[4] = (T)(a.trac_amp * sin(a.trac_omega * ts));
    }
    for (int c = 0; c < 6; ++c) a.sig[c * N + i] = s[c];
  }
  if (eval && a.epart) {
    __shared__ double red[256];
    red[threadIdx.x] = e_el;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
      if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
      __syncthreads();
    }
    if (threadIdx.x == 0) a.epart[blockIdx.x] = red[0];
  }
}

template <typename T>
__global__ void k_force(ElasticArgs<T> a) {
  if (ctrl_stopped(a.ctrl)) return;
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.N) return;
  const long N = a.N, sx = 1, sy = a.nx, sz = (long)a.nx * a.ny;
  const int x = (int)(i % a.nx), y = (int)((i / a.nx) % a.ny), z = (int)(i / ((long)a.nx * a.ny));
  const int stage = a.stage;
  T f[3];
  for (int r = 0; r < 3; ++r) {
    f[r] = d1(a.sig + voigt(r, 0) * N, i, x, a.nx, sx, a.dx) +
           d1(a.sig + voigt(r, 1) * N, i, y, a.ny, sy, a.dy) +
           d1(a.sig + voigt(r, 2) * N, i, z, a.nz, sz, a.dz);
  }
  const T* m = stage_in(a.tbl, stage);
  for (int s = 0; s < a.nsub; ++s) {
    if (!a.mel[s]) continue;
    const T* ms = m + (long)s * 3 * N;
    T mv[3], g[3][3];  // g[j][c] = d_j m_c
    for (int c = 0; c < 3; ++c) {
      mv[c] = ms[c * N + i];
      g[0][c] = d1(ms + c * N, i, x, a.nx, sx, a.dx);
      g[1][c] = d1(ms + c * N, i, y, a.ny, sy, a.dy);
      g[2][c] = d1(ms + c * N, i, z, a.nz, sz, a.dz);
    }
    for (int r = 0; r < 3; ++r) {
      T acc = T(2) * a.B1[s] * mv[r] * g[r][r];
      for (int j = 0; j < 3; ++j)
        if (j != r) acc += a.B2[s] * (mv[r] * g[j][j] + mv[j] * g[j][r]);
      f[r] += acc;
    }
  }
  const T* u = u_in(a.tbl, stage);
  const T* v = v_in(a.tbl, stage);
  T ku[3], kv[3];
  for (int c = 0; c < 3; ++c) {
    ku[c] = v[c * N + i];
    kv[c] = (f[c] - a.eta * ku[c]) * a.inv_rho;
  }
  T* KU = a.tbl->ku[stage - 1];
  T* KV = a.tbl->kv[stage - 1];
  for (int c = 0; c < 3; ++c) {
    KU[c * N + i] = ku[c];
    KV[c * N + i] = kv[c];
  }
  const double h = a.ctrl->h;
  const RKTab& rk = RK::t[a.tbl->rk];
  if (stage < a.tbl->ns) {
    T* uo = u_out(a.tbl, stage);
    T* vo = v_out(a.tbl, stage);
    const T* un = a.tbl->un;
    const T* vn = a.tbl->vn;
    for (int c = 0; c < 3; ++c) {
      T au = un[c * N + i], av = vn[c * N + i];
      for (int j = 0; j < stage - 1; ++j) {
        const T cj = (T)(rk.a[stage][j] * h);
        au += cj * a.tbl->ku[j][c * N + i];
        av += cj * a.tbl->kv[j][c * N + i];
      }
      const T cs = (T)(rk.a[stage][stage - 1] * h);
      uo[c * N + i] = au + cs * ku[c];
      vo[c * N + i] = av + cs * kv[c];
    }
  } else if (a.fuse2) {
    const T c21 = (T)(rk.a[1][0] * h);
    for (int c = 0; c < 3; ++c) {
      a.tbl->usa[c * N + i] = u[c * N + i] + c21 * ku[c];
      a.tbl->vsa[c * N + i] = v[c * N + i] + c21 * kv[c];
    }
  }
}

template <typename T>
__global__ void k_elastic_combine2(const Table<T>* tbl, const Ctrl* ctrl, long n3) {
  if (ctrl_stopped(ctrl)) return;
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n3) return;
  const T c = (T)(RK::t[tbl->rk].a[1][0] * ctrl->h);
  tbl->usa[i] = tbl->un[i] + c * tbl->ku[0][i];
  tbl->vsa[i] = tbl->vn[i] + c * tbl->kv[0][i];
}

template <typename T>
void launch_strain(const ElasticArgs<T>& a, hipStream_t st, Prof* prof) {
  ProfScope ps(prof, P_ELASTIC, st);
  hipLaunchKernelGGL(k_strain<T>, dim3((unsigned)((a.N + 255) / 256)), dim3(256), 0, st, a);
}

template <typename T>
void launch_elastic_stage(const ElasticArgs<T>& a, bool eval, hipStream_t st, Prof* prof) {
  ProfScope ps(prof, P_ELASTIC, st);
  const dim3 g((unsigned)((a.N + 255) / 256));
  hipLaunchKernelGGL(k_stress<T>, g, dim3(256), 0, st, a, eval ? 1 : 0);
  if (!eval) hipLaunchKernelGGL(k_force<T>, g, dim3(256), 0, st, a);
}

template <typename T>
void launch_elastic_combine2(const Table<T>* tbl, const Ctrl* ctrl, long N, hipStream_t st,
                             Prof* prof) {
  ProfScope ps(prof, P_COMBINE, st);
  hipLaunchKernelGGL(k_elastic_combine2<T>, dim3((unsigned)((3 * N + 255) / 256)), dim3(256), 0,
                     st, tbl, ctrl, 3 * N);
}

#define INST(T)                                                                        \
  template void launch_strain<T>(const ElasticArgs<T>&, hipStream_t, Prof*);          \
  template void launch_elastic_stage<T>(const ElasticArgs<T>&, bool, hipStream_t, Prof*); \
  template void launch_elastic_combine2<T>(const Table<T>*, const Ctrl*, long, hipStream_t, Prof*);
INST(float)
INST(double)

}  // namespace mmp
