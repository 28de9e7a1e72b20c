// Fused effective field + torque + Runge-Kutta stage kernel.
//
// One thread owns zc cells of an (x, y) column and marches along z with the
// z neighbours kept in registers; x/y neighbours come from global memory
// through L1/L2 (a 64x4 tile per block, blocks remapped so neighbouring
// tiles share an XCD's L2).  Shorter marches (small zc) give more waves to
// hide the latency of the dependent loads; longer ones re-read fewer
// z neighbours.  Per cell and sublattice it forms
//   B = B_demag + exchange (Eq. 3: 2A11/Ms lap m, A12/Ms lap m', 4A0/(Ms a^2) m')
//     + interfacial DMI (one sublattice) or homogeneous DMI d.(m1 x m2) (two)
//     + uniaxial/cubic anisotropy + Zeeman + B_mel (Eq. 9)
// and the torque tau = LLG (Eq. 2) + Zhang-Li, then, in a Runge-Kutta
// stage, writes k_s and immediately the next stage input
// y_{s+1} = normalise(y_n + h sum_j a_{s+1,j} k_j) (all point-wise), or at
// the last stage the FP64 error norm |sum_j e_j k_j| of the embedded pair in
// use (Table 2).
//
// Boundaries: a missing neighbour is the cell itself (Neumann), except in a
// layer with interfacial DMI, where the ghost is m -/+ d (dm/dn) with the
// natural boundary condition 2A dn m = -D (z x n) x m (Eq. 5 for one
// sublattice).  Zhang-Li uses clamped central differences.  Along a
// periodic axis (x or y) the neighbour of a boundary cell is the cell at the
// opposite end, for every stencil, and no boundary condition applies.
#include "field.h"

namespace mmp {

template <typename T>
__device__ __forceinline__ void cross3(const T* a, const T* b, T* o) {
  o[0] = a[1] * b[2] - a[2] * b[1];
  o[1] = a[2] * b[0] - a[0] * b[2];
  o[2] = a[0] * b[1] - a[1] * b[0];
}

// a*b - c*d with one rounding error (Kahan's difference of products)
template <typename T>
__device__ __forceinline__ T dop(T a, T b, T c, T d) {
  const T w = c * d;
  const T e = fma(-c, d, w);
  const T f = fma(a, b, -w);
  return f + e;
}

// m x m' accurate to a few ulp of the result even when m' ~ -m
template <typename T>
__device__ __forceinline__ void cross3_acc(const T* a, const T* b, T* o) {
  o[0] = dop(a[1], b[2], a[2], b[1]);
  o[1] = dop(a[2], b[0], a[0], b[2]);
  o[2] = dop(a[0], b[1], a[1], b[0]);
}

template <typename T>
__device__ __forceinline__ double dot3d(const T* a, const T* b) {
  return (double)a[0] * b[0] + (double)a[1] * b[1] + (double)a[2] * b[2];
}

// Ghosts beyond one face (axis ax, outward side +-1, cell size h) of every
// sublattice from the Neumann condition of Eq. 6:
//   2 A11^(s) g_s = A12 (g_s' x m_s) x m_s + m_s x w_s,  w_s = side W^(s)_ax,
// with (g x m) x m = -Q g, Q = I - m m^T; for two sublattices g2 solves
// (2 A2 I - A12^2/(2 A1) Q2 Q1) g2 = b2 - A12/(2 A1) Q2 b1 (Cramer's rule),
// then g1 = (b1 - A12 Q1 g2)/(2 A1).  A sublattice with A11 = 0 keeps a
// plain copy.  ghost = m + h g.
template <typename T, int NSUB>
__device__ void eq6_ghost(const FieldArgs<T>& a, const T (*m)[3], int ax, T side, T h,
                          T (*out)[3]) {
  T b[NSUB][3], g[NSUB][3];
#pragma unroll
  for (int s = 0; s < NSUB; ++s) {
    T w[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) w[c] = side * a.eW[s][ax][c];
    cross3(m[s], w, b[s]);
#pragma unroll
    for (int c = 0; c < 3; ++c) g[s][c] = T(0);
  }
  if constexpr (NSUB == 1) {
    if (a.eA[0] != T(0))
#pragma unroll
      for (int c = 0; c < 3; ++c) g[0][c] = b[0][c] / (T(2) * a.eA[0]);
  } else {
    const T A1 = a.eA[0], A2 = a.eA[1], A12 = a.eA12;
    if (A1 != T(0) && A2 != T(0)) {
      T Q1[3][3], Q2[3][3], M[3][3], r[3];
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          Q1[i][j] = (i == j ? T(1) : T(0)) - m[0][i] * m[0][j];
          Q2[i][j] = (i == j ? T(1) : T(0)) - m[1][i] * m[1][j];
        }
      const T c = A12 * A12 / (T(2) * A1), e = A12 / (T(2) * A1);
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        T q2b1 = T(0);
#pragma unroll
        for (int k = 0; k < 3; ++k) q2b1 += Q2[i][k] * b[0][k];
        r[i] = b[1][i] - e * q2b1;
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          T qq = T(0);
#pragma unroll
          for (int k = 0; k < 3; ++k) qq += Q2[i][k] * Q1[k][j];
          M[i][j] = (i == j ? T(2) * A2 : T(0)) - c * qq;
        }
      }
      const T det = M[0][0] * (M[1][1] * M[2][2] - M[1][2] * M[2][1]) -
                    M[0][1] * (M[1][0] * M[2][2] - M[1][2] * M[2][0]) +
                    M[0][2] * (M[1][0] * M[2][1] - M[1][1] * M[2][0]);
      const T id = T(1) / det;
      g[1][0] = id * (r[0] * (M[1][1] * M[2][2] - M[1][2] * M[2][1]) -
                      M[0][1] * (r[1] * M[2][2] - M[1][2] * r[2]) +
                      M[0][2] * (r[1] * M[2][1] - M[1][1] * r[2]));
      g[1][1] = id * (M[0][0] * (r[1] * M[2][2] - M[1][2] * r[2]) -
                      r[0] * (M[1][0] * M[2][2] - M[1][2] * M[2][0]) +
                      M[0][2] * (M[1][0] * r[2] - r[1] * M[2][0]));
      g[1][2] = id * (M[0][0] * (M[1][1] * r[2] - r[1] * M[2][1]) -
                      M[0][1] * (M[1][0] * r[2] - r[1] * M[2][0]) +
                      r[0] * (M[1][0] * M[2][1] - M[1][1] * M[2][0]));
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        T q1g2 = T(0);
#pragma unroll
        for (int k = 0; k < 3; ++k) q1g2 += Q1[i][k] * g[1][k];
        g[0][i] = (b[0][i] - A12 * q1g2) / (T(2) * A1);
      }
    } else if (A1 != T(0)) {
#pragma unroll
      for (int c = 0; c < 3; ++c) g[0][c] = b[0][c] / (T(2) * A1);
    } else if (A2 != T(0)) {
#pragma unroll
      for (int c = 0; c < 3; ++c) g[1][c] = b[1][c] / (T(2) * A2);
    }
  }
#pragma unroll
  for (int s = 0; s < NSUB; ++s)
#pragma unroll
    for (int c = 0; c < 3; ++c) out[s][c] = m[s][c] + h * g[s][c];
}

// Block w (tile-major over z chunks) of one grid; stage and fuse2 come from
// the launch so that one argument block serves every stage.
// GDMI: general DMI tensors with the Eq. 6 ghosts on every stencil.
// GBX: exchange links between different grains scaled by gbx_scale.
template <typename T, int NSUB, bool EVAL, bool GDMI = false, bool GBX = false>
__device__ __forceinline__ void field_block(const FieldArgs<T>& a, const int w, const int stage,
                                            const int fuse2) {
  const int ntile = a.nbx * a.nby;
  if (w >= ntile * a.nzc) return;
  const int tile = w % ntile;
  const int z0 = (w / ntile) * a.zc;
  const int z1 = min(a.nz, z0 + a.zc);
  const int x = (tile % a.nbx) * kTileX + (int)(threadIdx.x % kTileX);
  const int y = (tile / a.nbx) * kTileY + (int)(threadIdx.x / kTileX);
  const bool in = x < a.nx && y < a.ny;
  const long N = a.N;
  const long N3 = 3 * N;
  const gcptr<T> m = (gcptr<T>)(EVAL ? a.tbl->yn : stage_in(a.tbl, stage));

  double h = 0.0;
  int ns = 0;
  T ca[6] = {0, 0, 0, 0, 0, 0};
  double ew[7] = {0, 0, 0, 0, 0, 0, 0};
  gcptr<T> kin[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  gptr<T> kout = nullptr;
  gptr<T> ynext = nullptr;
  gcptr<T> yn = nullptr;
  if (!EVAL) {
    h = a.ctrl->h;
    ns = a.tbl->ns;
    const RKTab& rk = RK::t[a.tbl->rk];
    kout = (gptr<T>)a.tbl->k[stage - 1];
    yn = (gcptr<T>)a.tbl->yn;
    for (int j = 0; j < stage - 1; ++j) kin[j] = (gcptr<T>)a.tbl->k[j];
    if (stage < ns) {
      ynext = (gptr<T>)stage_out(a.tbl, stage);
      for (int j = 0; j < stage; ++j) ca[j] = (T)(rk.a[stage][j] * h);
    } else {
      if (fuse2) ynext = (gptr<T>)a.tbl->sa;
      ca[0] = (T)(rk.a[1][0] * h);
      for (int j = 0; j < ns - 1; ++j) kin[j] = (gcptr<T>)a.tbl->k[j];
      for (int j = 0; j < ns; ++j) ew[j] = rk.e[j];
    }
  }
  // slopes the one-sublattice march loads up front (see below): the ones
  // this stage sums, and in the other slots a buffer read anyway (k_1, or
  // y_n at stage 1, which has no earlier slope; never a null table entry)
  const gcptr<T> spare = stage >= 2 ? kin[0] : yn;
  gcptr<T> kslot[6];
  for (int j = 0; j < 6; ++j) {
    const bool used = !EVAL && (stage < ns ? j < stage - 1 : (j < ns - 1 && ew[j] != 0.0));
    kslot[j] = used ? kin[j] : spare;
  }
  const gcptr<T> yslot = stage < ns ? yn : spare;

  double eacc[kNE];
  for (int t = 0; t < kNE; ++t) eacc[t] = 0.0;
  double emax = 0.0;

  if (in) {
    T cur[NSUB][3], zm[NSUB][3], zp[NSUB][3];
    const long col = (long)y * a.nx + x;
    const long plane = (long)a.nx * a.ny;
    const long i0 = (long)z0 * plane + col;
    // A missing neighbour is the cell itself, so every neighbour load is an
    // unconditional load from a clamped offset: no branches between the
    // loads, which then all go out before the first wait.
    // (on a periodic axis the cell at the opposite end)
    const long dxm = x > 0 ? -1 : (a.per_x ? a.nx - 1 : 0);
    const long dxp = x + 1 < a.nx ? 1 : (a.per_x ? 1 - a.nx : 0);
    const long dym = y > 0 ? -(long)a.nx : (a.per_y ? (long)(a.ny - 1) * a.nx : 0);
    const long dyp = y + 1 < a.ny ? (long)a.nx : (a.per_y ? -(long)(a.ny - 1) * a.nx : 0);
    const long dz0 = z0 > 0 ? -plane : 0;
#pragma unroll
    for (int s = 0; s < NSUB; ++s)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        cur[s][c] = m[s * N3 + c * N + i0];
        zm[s][c] = m[s * N3 + c * N + i0 + dz0];
      }
    for (int z = z0; z < z1; ++z) {
      const long i = (long)z * plane + col;
      const long dzp = z + 1 < a.nz ? plane : 0;
      // one sublattice: the stage slopes and y_n of this cell are requested
      // with the stencil loads (they do not depend on the field, and loaded
      // after the k_s stores below they would wait for a second round trip)
      // Every slot is loaded (a slot this stage does not use reads k_1
      // again, a cache hit): no branch between the loads, which then all go
      // out before the first wait.
      T kv1[6][3], yv1[3];
      if constexpr (NSUB == 1 && !EVAL) {
        if (stage < ns || !fuse2) {
#pragma unroll
          for (int j = 0; j < 6; ++j)
#pragma unroll
            for (int c = 0; c < 3; ++c) kv1[j][c] = kslot[j][i + c * N];
#pragma unroll
          for (int c = 0; c < 3; ++c) yv1[c] = yslot[i + c * N];
        }
      }
#pragma unroll
      for (int s = 0; s < NSUB; ++s)
#pragma unroll
        for (int c = 0; c < 3; ++c) zp[s][c] = m[s * N3 + c * N + i + dzp];
      T xm[NSUB][3], xp[NSUB][3], ym[NSUB][3], yp[NSUB][3];
#pragma unroll
      for (int s = 0; s < NSUB; ++s)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const gcptr<T> mc = m + s * N3 + c * N + i;
          xm[s][c] = mc[dxm];
          xp[s][c] = mc[dxp];
          ym[s][c] = mc[dym];
          yp[s][c] = mc[dyp];
        }
      T Bd[3] = {0, 0, 0};
      if (a.has_demag) {
        Bd[0] = ntload(a.Bd + i);
        Bd[1] = ntload(a.Bd + N + i);
        Bd[2] = ntload(a.Bd + 2 * N + i);
      }
      T ep[6] = {0, 0, 0, 0, 0, 0};
      if (a.has_mel) {
#pragma unroll
        for (int c = 0; c < 6; ++c) ep[c] = a.eps[c * N + i];
      }
      T uax[3];
      if (a.has_anis_u && a.grain) {
        const int g = a.grain[i];
        uax[0] = a.gaxes[3 * g];
        uax[1] = a.gaxes[3 * g + 1];
        uax[2] = a.gaxes[3 * g + 2];
      }
      // link weights x-, x+, y-, y+, z-, z+ of the A11 and A12 stencils: the
      // scale across a grain boundary, 1 inside a grain and towards a
      // missing neighbour (its offset is 0, the cell's own grain)
      T wl[6];
      if constexpr (GBX) {
        const uint16_t* gr = a.grain + i;
        const int g0 = gr[0];
        const T f = a.gbx_scale;
        wl[0] = gr[dxm] == g0 ? T(1) : f;
        wl[1] = gr[dxp] == g0 ? T(1) : f;
        wl[2] = gr[dym] == g0 ? T(1) : f;
        wl[3] = gr[dyp] == g0 ? T(1) : f;
        wl[4] = gr[z > 0 ? -plane : 0] == g0 ? T(1) : f;
        wl[5] = gr[dzp] == g0 ? T(1) : f;
      }
      auto lk = [&](int k, T v) -> T {
        if constexpr (GBX) return wl[k] * v;
        else return v;
      };
      const bool dmil = NSUB == 1 && a.has_dmi && (a.dmi_layer < 0 || z == a.dmi_layer);
      // neighbours seen by the exchange and DMI stencils: the loaded ones, or
      // the Eq. 6 ghosts on the faces of the open axes (z neighbours are
      // copied: the rotating z registers must keep the cells themselves)
      T sxm[NSUB][3], sxp[NSUB][3], sym[NSUB][3], syp[NSUB][3], szm[NSUB][3], szp[NSUB][3];
#pragma unroll
      for (int s = 0; s < NSUB; ++s)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          sxm[s][c] = xm[s][c]; sxp[s][c] = xp[s][c]; sym[s][c] = ym[s][c];
          syp[s][c] = yp[s][c]; szm[s][c] = zm[s][c]; szp[s][c] = zp[s][c];
        }
      if constexpr (GDMI) {
        if (x == 0 && !a.per_x) eq6_ghost<T, NSUB>(a, cur, 0, T(-1), a.dx, sxm);
        if (x + 1 == a.nx && !a.per_x) eq6_ghost<T, NSUB>(a, cur, 0, T(1), a.dx, sxp);
        if (y == 0 && !a.per_y) eq6_ghost<T, NSUB>(a, cur, 1, T(-1), a.dy, sym);
        if (y + 1 == a.ny && !a.per_y) eq6_ghost<T, NSUB>(a, cur, 1, T(1), a.dy, syp);
        if (z == 0) eq6_ghost<T, NSUB>(a, cur, 2, T(-1), a.dz, szm);
        if (z + 1 == a.nz) eq6_ghost<T, NSUB>(a, cur, 2, T(1), a.dz, szp);
      }

#pragma unroll
      for (int s = 0; s < NSUB; ++s) {
        const SubC<T>& C = a.sc[s];
        const T* mm = cur[s];
        // ghosted in-plane neighbours for exchange/DMI
        T gxm[3], gxp[3], gym[3], gyp[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          gxm[c] = sxm[s][c]; gxp[c] = sxp[s][c]; gym[c] = sym[s][c]; gyp[c] = syp[s][c];
        }
        if (dmil) {
          // boundary condition of Eq. 5 on the faces of the open axes
          const T k = C.kdmi;
          if (x == 0 && !a.per_x) {
            gxm[0] = mm[0] - a.dx * k * mm[2]; gxm[1] = mm[1]; gxm[2] = mm[2] + a.dx * k * mm[0];
          }
          if (x + 1 == a.nx && !a.per_x) {
            gxp[0] = mm[0] + a.dx * k * mm[2]; gxp[1] = mm[1]; gxp[2] = mm[2] - a.dx * k * mm[0];
          }
          if (y == 0 && !a.per_y) {
            gym[0] = mm[0]; gym[1] = mm[1] - a.dy * k * mm[2]; gym[2] = mm[2] + a.dy * k * mm[1];
          }
          if (y + 1 == a.ny && !a.per_y) {
            gyp[0] = mm[0]; gyp[1] = mm[1] + a.dy * k * mm[2]; gyp[2] = mm[2] - a.dy * k * mm[1];
          }
        }
        T B[3] = {0, 0, 0};     // field driving the torque (all but A0)
        T Bout[3] = {0, 0, 0};  // extra output-only part (A0, eval mode)
        bool a0_on = false;
        T bt[3];
        auto add = [&](int term, const T* b) {
          if (!EVAL || (a.mask & (1u << term))) {
            B[0] += b[0]; B[1] += b[1]; B[2] += b[2];
          }
        };
        // exchange
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const T l = (lk(0, gxm[c] - mm[c]) + lk(1, gxp[c] - mm[c])) * a.idx2 +
                      (lk(2, gym[c] - mm[c]) + lk(3, gyp[c] - mm[c])) * a.idy2 +
                      (lk(4, szm[s][c] - mm[c]) + lk(5, szp[s][c] - mm[c])) * a.idz2;
          bt[c] = C.cex * l;
        }
        add(1, bt);
        if (EVAL) eacc[1] += -0.5 * C.Ms_d * dot3d(mm, bt);
        // interfacial DMI
        if (dmil) {
          bt[0] = C.cdmi * ((gxp[2] - gxm[2]) * a.i2dx);
          bt[1] = C.cdmi * ((gyp[2] - gym[2]) * a.i2dy);
          bt[2] = -C.cdmi * ((gxp[0] - gxm[0]) * a.i2dx + (gyp[1] - gym[1]) * a.i2dy);
          add(4, bt);
          if (EVAL) eacc[4] += -0.5 * C.Ms_d * dot3d(mm, bt);
        }
        // DMI tensors (Eq. 4): B = sum_i d_i m x cW_i + d_i m' x cW'_i,
        // cW = -2 W/Ms, central differences over the Eq. 6 ghosts
        if constexpr (GDMI) {
          T dm[3][3], dmo[3][3];
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            dm[0][c] = (sxp[s][c] - sxm[s][c]) * a.i2dx;
            dm[1][c] = (syp[s][c] - sym[s][c]) * a.i2dy;
            dm[2][c] = (szp[s][c] - szm[s][c]) * a.i2dz;
            if (NSUB == 2) {
              const int o = 1 - s;
              dmo[0][c] = (sxp[o][c] - sxm[o][c]) * a.i2dx;
              dmo[1][c] = (syp[o][c] - sym[o][c]) * a.i2dy;
              dmo[2][c] = (szp[o][c] - szm[o][c]) * a.i2dz;
            }
          }
          T acc[3] = {0, 0, 0}, tmp[3];
#pragma unroll
          for (int i = 0; i < 3; ++i) {
            cross3(dm[i], a.cW[s][i], tmp);
            acc[0] += tmp[0]; acc[1] += tmp[1]; acc[2] += tmp[2];
            if (NSUB == 2) {
              cross3(dmo[i], a.cW12[s][i], tmp);
              acc[0] += tmp[0]; acc[1] += tmp[1]; acc[2] += tmp[2];
            }
          }
          add(4, acc);
          if (EVAL) eacc[4] += -0.5 * C.Ms_d * dot3d(mm, acc);
        }
        // inter-sublattice exchange (Eq. 3) with every other sublattice:
        // A12/Ms lap m' (inhomogeneous) and 4 A0/(Ms a^2) m' (homogeneous)
        if (NSUB >= 2) {
#pragma unroll
          for (int c = 0; c < 3; ++c) bt[c] = T(0);
#pragma unroll
          for (int o = 0; o < NSUB; ++o) {
            if (o == s) continue;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
              const T mo = cur[o][c];
              const T l = (lk(0, sxm[o][c] - mo) + lk(1, sxp[o][c] - mo)) * a.idx2 +
                          (lk(2, sym[o][c] - mo) + lk(3, syp[o][c] - mo)) * a.idy2 +
                          (lk(4, szm[o][c] - mo) + lk(5, szp[o][c] - mo)) * a.idz2;
              bt[c] += C.cnn * l;
            }
          }
          add(2, bt);
          if (EVAL) eacc[2] += -0.5 * C.Ms_d * dot3d(mm, bt);
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            T so = T(0);
#pragma unroll
            for (int o = 0; o < NSUB; ++o)
              if (o != s) so += cur[o][c];
            bt[c] = C.ccell * so;
          }
          // The homogeneous inter-sublattice field is ~1000x larger than the
          // torque it leaves when m' ~ -m, so its torque is formed from an
          // accurate m x m' (tau is linear in B) instead of from B.
          if (!EVAL || (a.mask & (1u << 3))) {
            a0_on = true;
            if (EVAL) {
              Bout[0] += bt[0]; Bout[1] += bt[1]; Bout[2] += bt[2];
            }
          }
          if (EVAL) eacc[3] += -0.5 * C.Ms_d * dot3d(mm, bt);
          // homogeneous DMI d.(m1 x m2): B = m' x dh, dh = -/+ d/Ms
          if (NSUB == 2 && a.has_dmih) {
            cross3(cur[1 - s], C.dh, bt);
            add(4, bt);
            if (EVAL) eacc[4] += -0.5 * C.Ms_d * dot3d(mm, bt);
          }
        }
        // demag
        if (a.has_demag && C.nonzero) {
          add(0, Bd);
          if (EVAL) eacc[0] += -0.5 * C.Ms_d * dot3d(mm, Bd);
        }
        // uniaxial anisotropy
        if (a.has_anis_u) {
          const T* u = a.grain ? uax : C.u;
          const T um = u[0] * mm[0] + u[1] * mm[1] + u[2] * mm[2];
          const T f = C.cku1 * um + C.cku2 * um * um * um;
          bt[0] = f * u[0]; bt[1] = f * u[1]; bt[2] = f * u[2];
          add(5, bt);
          if (EVAL && C.nonzero) {
            const double umd = (double)um;
            eacc[5] += -C.Ku1_d * umd * umd - C.Ku2_d * umd * umd * umd * umd;
          }
        }
        // cubic anisotropy
        if (a.has_anis_c) {
          const T a1 = C.c1[0] * mm[0] + C.c1[1] * mm[1] + C.c1[2] * mm[2];
          const T a2 = C.c2[0] * mm[0] + C.c2[1] * mm[1] + C.c2[2] * mm[2];
          const T a3 = C.c3[0] * mm[0] + C.c3[1] * mm[1] + C.c3[2] * mm[2];
          const T f1 = -C.ckc * a1 * (a2 * a2 + a3 * a3);
          const T f2 = -C.ckc * a2 * (a1 * a1 + a3 * a3);
          const T f3 = -C.ckc * a3 * (a1 * a1 + a2 * a2);
#pragma unroll
          for (int c = 0; c < 3; ++c) bt[c] = f1 * C.c1[c] + f2 * C.c2[c] + f3 * C.c3[c];
          add(6, bt);
          if (EVAL && C.nonzero) {
            const double d1 = a1, d2 = a2, d3 = a3;
            eacc[6] += C.Kc1_d * (d1 * d1 * d2 * d2 + d2 * d2 * d3 * d3 + d3 * d3 * d1 * d1);
          }
        }
        // Zeeman
        add(7, a.bext);
        if (EVAL) eacc[7] += -C.Ms_d * dot3d(mm, a.bext);
        // magnetoelastic field
        if (a.has_mel) {
          bt[0] = -(C.cmel1 * ep[0] * mm[0] + C.cmel2 * (ep[3] * mm[1] + ep[4] * mm[2]));
          bt[1] = -(C.cmel1 * ep[1] * mm[1] + C.cmel2 * (ep[3] * mm[0] + ep[5] * mm[2]));
          bt[2] = -(C.cmel1 * ep[2] * mm[2] + C.cmel2 * (ep[4] * mm[0] + ep[5] * mm[1]));
          add(8, bt);
          if (EVAL && C.nonzero) {
            const double m0 = mm[0], m1 = mm[1], m2 = mm[2];
            eacc[8] += C.B1_d * ((double)ep[0] * m0 * m0 + (double)ep[1] * m1 * m1 +
                                 (double)ep[2] * m2 * m2) +
                       2.0 * C.B2_d * ((double)ep[3] * m0 * m1 + (double)ep[4] * m0 * m2 +
                                       (double)ep[5] * m1 * m2);
          }
        }
        // torque
        T mxB[3], mxmxB[3], tau[3];
        cross3(mm, B, mxB);
        cross3(mm, mxB, mxmxB);
#pragma unroll
        for (int c = 0; c < 3; ++c) tau[c] = -C.gl * (mxB[c] + C.alpha * mxmxB[c]);
        if (NSUB >= 2 && a0_on) {
          T w[3] = {0, 0, 0}, mxw[3];
#pragma unroll
          for (int o = 0; o < NSUB; ++o) {
            if (o == s) continue;
            T wo[3];
            cross3_acc(mm, cur[o], wo);
            w[0] += wo[0]; w[1] += wo[1]; w[2] += wo[2];
          }
          cross3(mm, w, mxw);
#pragma unroll
          for (int c = 0; c < 3; ++c) tau[c] -= C.gl * C.ccell * (w[c] + C.alpha * mxw[c]);
        }
        const bool zl = EVAL ? (a.add_zl && C.has_zl) : C.has_zl;
        if (zl) {
          T dm[3], mxdm[3], mxmxdm[3];
#pragma unroll
          for (int c = 0; c < 3; ++c)
            dm[c] = C.zu[0] * (xp[s][c] - xm[s][c]) * a.i2dx +
                    C.zu[1] * (yp[s][c] - ym[s][c]) * a.i2dy +
                    C.zu[2] * (zp[s][c] - zm[s][c]) * a.i2dz;
          cross3(mm, dm, mxdm);
          cross3(mm, mxdm, mxmxdm);
#pragma unroll
          for (int c = 0; c < 3; ++c) tau[c] -= C.zla * mxmxdm[c] + C.zlb * mxdm[c];
        }
        const long base = s * N3 + i;
        if (EVAL) {
          if (a.bout) {
            if (a.out_torque) {
              a.bout[base] = tau[0];
              a.bout[base + N] = tau[1];
              a.bout[base + 2 * N] = tau[2];
            } else {
              a.bout[base] = B[0] + Bout[0];
              a.bout[base + N] = B[1] + Bout[1];
              a.bout[base + 2 * N] = B[2] + Bout[2];
            }
          }
        } else {
          if (!(isfinite(tau[0]) && isfinite(tau[1]) && isfinite(tau[2])))
            atomicOr(&a.ctrl->nonfinite, 1);
          kout[base] = tau[0];
          kout[base + N] = tau[1];
          kout[base + 2 * N] = tau[2];
          if (stage < ns) {
            T v[3];
            if constexpr (NSUB == 1) {
              // the slopes this stage needs, loaded at the top of the
              // iteration, summed in order.  (Two sublattices would need
              // twice the registers and lose more waves than the batching
              // gains.)
#pragma unroll
              for (int c = 0; c < 3; ++c) {
                T acc = yv1[c];
#pragma unroll
                for (int j = 0; j < 5; ++j)
                  if (j < stage - 1) acc += ca[j] * kv1[j][c];
                acc += ca[stage - 1] * tau[c];
                v[c] = acc;
              }
            } else {
#pragma unroll
              for (int c = 0; c < 3; ++c) {
                T acc = yn[base + c * N];
                for (int j = 0; j < stage - 1; ++j) acc += ca[j] * kin[j][base + c * N];
                acc += ca[stage - 1] * tau[c];
                v[c] = acc;
              }
            }
            const T inv = T(1) / sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
            ynext[base] = v[0] * inv;
            ynext[base + N] = v[1] * inv;
            ynext[base + 2 * N] = v[2] * inv;
          } else if (!fuse2) {
            // error weights: e_j of the earlier slopes (zero weights skip
            // their loads), then e_ns of this stage's own slope
            double ev[3];
            if constexpr (NSUB == 1) {
#pragma unroll
              for (int c = 0; c < 3; ++c) {
                double acc = 0.0;
#pragma unroll
                for (int j = 0; j < 6; ++j)
                  if (j < ns - 1 && ew[j] != 0.0) acc += ew[j] * (double)kv1[j][c];
                ev[c] = acc + ew[ns - 1] * (double)tau[c];
              }
            } else {
#pragma unroll
              for (int c = 0; c < 3; ++c) {
                double acc = 0.0;
                for (int j = 0; j < ns - 1; ++j)
                  if (ew[j] != 0.0) acc += ew[j] * (double)kin[j][base + c * N];
                ev[c] = acc + ew[ns - 1] * (double)tau[c];
              }
            }
            const double nrm = sqrt(ev[0] * ev[0] + ev[1] * ev[1] + ev[2] * ev[2]);
            emax = nrm > emax ? nrm : emax;
          } else {
            {
              T v[3];
#pragma unroll
              for (int c = 0; c < 3; ++c) v[c] = mm[c] + ca[0] * tau[c];
              const T inv = T(1) / sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
              ynext[base] = v[0] * inv;
              ynext[base + N] = v[1] * inv;
              ynext[base + 2 * N] = v[2] * inv;
            }
          }
        }
      }
#pragma unroll
      for (int s = 0; s < NSUB; ++s)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          zm[s][c] = cur[s][c];
          cur[s][c] = zp[s][c];
        }
    }
  }

  if (EVAL) {
    if (a.epart) {
      __shared__ double red[kNE][256];
      for (int t = 0; t < kNE; ++t) red[t][threadIdx.x] = eacc[t] * a.V;
      __syncthreads();
      for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st)
          for (int t = 0; t < kNE; ++t) red[t][threadIdx.x] += red[t][threadIdx.x + st];
        __syncthreads();
      }
      if (threadIdx.x < kNE) a.epart[(long)w * kNE + threadIdx.x] = red[threadIdx.x][0];
    }
  } else if (stage == ns && !fuse2) {
    __shared__ double red[256];
    red[threadIdx.x] = emax;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
      if ((int)threadIdx.x < st) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + st]);
      __syncthreads();
    }
    if (threadIdx.x == 0) a.errpart[w] = red[0];
  }
}

template <typename T, int NSUB, bool EVAL, bool GDMI = false, bool GBX = false>
__global__ __launch_bounds__(256) void k_field(const FieldArgs<T> a) {
  if (ctrl_stopped(a.ctrl)) return;
  field_block<T, NSUB, EVAL, GDMI, GBX>(a, xcd_remap(blockIdx.x, a.nb_pad), a.stage, a.fuse2);
}

// Many grids in one launch: block b runs block work[b].y of grid work[b].x
// (the argument blocks live in device memory); a grid whose run is over
// skips its blocks.
template <typename T, int NSUB>
__global__ __launch_bounds__(256) void k_field_multi(const FieldArgs<T>* __restrict__ args,
                                                     const int2* __restrict__ work, int nwork,
                                                     int nb_pad, int stage, int fuse2) {
  const int b = xcd_remap(blockIdx.x, nb_pad);
  if (b >= nwork) return;
  const int2 wk = work[b];
  const FieldArgs<T>& a = args[wk.x];
  if (ctrl_stopped(a.ctrl)) return;
  field_block<T, NSUB, false>(a, wk.y, stage, fuse2);
}

template <typename T>
void launch_field_multi(const FieldArgs<T>* args, const int2* work, int nwork, int nsub, int stage,
                        int fuse2, hipStream_t st) {
  const int nb_pad = round_up(nwork, 8);
  if (nsub == 1)
    hipLaunchKernelGGL((k_field_multi<T, 1>), dim3(nb_pad), dim3(256), 0, st, args, work, nwork,
                       nb_pad, stage, fuse2);
  else
    hipLaunchKernelGGL((k_field_multi<T, 2>), dim3(nb_pad), dim3(256), 0, st, args, work, nwork,
                       nb_pad, stage, fuse2);
}

// The Eq. 6 ghosts (GDMI) exist for one and two sublattices only.
template <typename T, bool EVAL, bool GDMI, bool GBX>
void launch_field_nsub(const FieldArgs<T>& a, hipStream_t st) {
  const dim3 g(a.nb_pad), b(256);
  if (a.nsub == 1) {
    hipLaunchKernelGGL((k_field<T, 1, EVAL, GDMI, GBX>), g, b, 0, st, a);
  } else if (a.nsub == 2) {
    hipLaunchKernelGGL((k_field<T, 2, EVAL, GDMI, GBX>), g, b, 0, st, a);
  } else if constexpr (!GDMI) {
    hipLaunchKernelGGL((k_field<T, 3, EVAL, GDMI, GBX>), g, b, 0, st, a);
  }
}

template <typename T, bool EVAL>
void launch_field_var(const FieldArgs<T>& a, hipStream_t st) {
  if (a.gdmi) {
    if (a.gbx) launch_field_nsub<T, EVAL, true, true>(a, st);
    else launch_field_nsub<T, EVAL, true, false>(a, st);
  } else {
    if (a.gbx) launch_field_nsub<T, EVAL, false, true>(a, st);
    else launch_field_nsub<T, EVAL, false, false>(a, st);
  }
}

template <typename T>
void launch_field(const FieldArgs<T>& a, bool eval, hipStream_t st, Prof* prof) {
  ProfScope ps(prof, P_FIELD, st);
  if (eval) launch_field_var<T, true>(a, st);
  else launch_field_var<T, false>(a, st);
}

// --------------------------------------------------------- combine2 ----
// Stage-2 input for a new attempt: normalise(y_n + h a21 k1).
template <typename T>
__device__ __forceinline__ void combine2_cell(const Table<T>* tbl, const Ctrl* ctrl, long Ncell,
                                              long i) {
  const long s = i / Ncell, cell = i - s * Ncell;
  const long base = s * 3 * Ncell + cell;
  const T c = (T)(RK::t[tbl->rk].a[1][0] * ctrl->h);
  const gcptr<T> yn = (gcptr<T>)tbl->yn;
  const gcptr<T> k1 = (gcptr<T>)tbl->k[0];
  T v[3];
  for (int q = 0; q < 3; ++q) v[q] = yn[base + q * Ncell] + c * k1[base + q * Ncell];
  const T inv = T(1) / sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
  const gptr<T> o = (gptr<T>)tbl->sa;
  for (int q = 0; q < 3; ++q) o[base + q * Ncell] = v[q] * inv;
}

template <typename T>
__global__ void k_combine2_cells(const Table<T>* tbl, const Ctrl* ctrl, long Ncell, int nsub) {
  if (ctrl_stopped(ctrl)) return;
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= Ncell * nsub) return;
  combine2_cell<T>(tbl, ctrl, Ncell, i);
}

template <typename T>
void launch_combine2(const Table<T>* tbl, const Ctrl* ctrl, long Ncell, int nsub, hipStream_t st,
                     Prof* prof) {
  ProfScope ps(prof, P_COMBINE, st);
  const long n = Ncell * nsub;
  hipLaunchKernelGGL((k_combine2_cells<T>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
                     tbl, ctrl, Ncell, nsub);
}

// ---------------------------------------------------------- control ----
template <typename T>
__device__ __forceinline__ void control_block(Ctrl* c, Table<T>* tbl, const double* errpart,
                                              int nerr, int elastic) {
  if (c->done || c->status) return;
  __shared__ double red[256];
  double e = 0.0;
  if (!c->fixed)
    for (int i = threadIdx.x; i < nerr; i += blockDim.x) e = fmax(e, errpart[i]);
  red[threadIdx.x] = e;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  if (c->nonfinite) {
    c->status = MMP_E_NONFINITE;
    c->done = 1;
    return;
  }
  const double h = c->h;
  const double err = c->fixed ? 0.0 : h * red[0];
  c->err = err;
  const bool acc = c->fixed || err <= c->tol;
  c->accepted = acc ? 1 : 0;
  if (acc) {
    T* t;
    t = tbl->yn; tbl->yn = tbl->ynew; tbl->ynew = t;
    // the last stage's slope (at y_{n+1}) is the next step's k_1
    const int l = tbl->ns - 1;
    t = tbl->k[0]; tbl->k[0] = tbl->k[l]; tbl->k[l] = t;
    if (elastic) {
      t = tbl->un; tbl->un = tbl->unew; tbl->unew = t;
      t = tbl->vn; tbl->vn = tbl->vnew; tbl->vnew = t;
      t = tbl->ku[0]; tbl->ku[0] = tbl->ku[l]; tbl->ku[l] = t;
      t = tbl->kv[0]; tbl->kv[0] = tbl->kv[l]; tbl->kv[l] = t;
    }
    c->steps += 1;
    if (c->fixed) {
      c->sample_k += 1;  // counts steps of this segment
      c->t = c->t0 + (double)c->sample_k * h;
      if (c->max_attempts > 0 && c->sample_k >= c->max_attempts) c->done = 1;
    } else {
      c->t = c->land ? fmin(c->t_next, c->t_end) : c->t + h;
      if (c->land && c->sample_every > 0.0 && c->t == c->t_next) {
        c->sample_pending = 1;
        c->sample_k += 1;
        c->t_next = c->t0 + (double)c->sample_k * c->sample_every;
        // an output time a few ulp short of t_end is t_end itself
        if (c->t_next >= c->t_end - 1e-9 * (c->t_end - c->t0)) c->t_next = c->t_end;
      }
      if (c->t >= c->t_end) c->done = 1;
    }
  } else {
    c->rejects += 1;
  }
  if (!c->fixed) {
    double fac = c->fac_max;
    if (err > 0.0) fac = c->safety * pow(c->tol / err, 1.0 / (RK::t[tbl->rk].q + 1));
    fac = fmin(c->fac_max, fmax(c->fac_min, fac));
    c->dt = h * fac;
    if (c->dt_max > 0.0) c->dt = fmin(c->dt, c->dt_max);
    if (c->dt < c->dt_min) {
      c->status = MMP_E_DT_UNDERFLOW;
      c->done = 1;
    }
    if (c->max_attempts > 0 && c->steps + c->rejects >= c->max_attempts) c->done = 1;
    const double target = fmin(c->t_next, c->t_end);
    const double rem = target - c->t;
    c->land = c->dt >= rem ? 1 : 0;
    c->h = c->land ? rem : c->dt;
  }
}

template <typename T>
__global__ void k_control(Ctrl* c, Table<T>* tbl, const double* errpart, int nerr, int elastic) {
  control_block<T>(c, tbl, errpart, nerr, elastic);
}

// one block per grid of a batch
template <typename T>
__global__ void k_control_multi(const StepWork<T>* __restrict__ w) {
  const StepWork<T> g = w[blockIdx.x];
  control_block<T>(g.ctrl, g.tbl, g.errpart, g.nerr, 0);
}

template <typename T>
__global__ void k_combine2_multi(const StepWork<T>* __restrict__ w) {
  const StepWork<T> g = w[blockIdx.y];
  if (ctrl_stopped(g.ctrl)) return;
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.N * g.nsub) return;
  combine2_cell<T>(g.tbl, g.ctrl, g.N, i);
}

template <typename T>
void launch_step_multi(const StepWork<T>* w, int ngrids, long max_cells, hipStream_t st) {
  hipLaunchKernelGGL((k_control_multi<T>), dim3(ngrids), dim3(256), 0, st, w);
  hipLaunchKernelGGL((k_combine2_multi<T>), dim3((unsigned)((max_cells + 255) / 256), ngrids),
                     dim3(256), 0, st, w);
}

template <typename T>
void launch_control(Ctrl* ctrl, Table<T>* tbl, const double* errpart, int nerr, int elastic,
                    hipStream_t st, Prof* prof) {
  ProfScope ps(prof, P_CONTROL, st);
  hipLaunchKernelGGL((k_control<T>), dim3(1), dim3(256), 0, st, ctrl, tbl, errpart, nerr, elastic);
}

// ----------------------------------------------------------- sampling --
template <typename T>
__global__ void k_sample_part(const Ctrl* c, const Table<T>* tbl, int nsub, long N, double* part) {
  if (!c->sample_pending) return;
  __shared__ double red[9][256];
  double acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  const T* y = tbl->yn;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (long)gridDim.x * blockDim.x)
    for (int s = 0; s < nsub; ++s)
      for (int q = 0; q < 3; ++q) acc[s * 3 + q] += (double)y[(s * 3 + q) * N + i];
  for (int q = 0; q < 9; ++q) red[q][threadIdx.x] = acc[q];
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st)
      for (int q = 0; q < 9; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x < 9) part[blockIdx.x * 9 + threadIdx.x] = red[threadIdx.x][0];
}

__global__ void k_sample_final(Ctrl* c, const double* part, int nblk, long N, int nsub,
                               double* sample_t, double* sample_m, int cap) {
  if (!c->sample_pending) return;
  if (threadIdx.x != 0) return;
  const int k = c->nsamples;
  if (k < cap) {
    sample_t[k] = c->t;
    for (int q = 0; q < 3 * nsub; ++q) {
      double acc = 0.0;
      for (int b = 0; b < nblk; ++b) acc += part[b * 9 + q];
      sample_m[k * 3 * nsub + q] = acc / (double)N;
    }
  }
  c->nsamples = k + 1;
  c->sample_pending = 0;
}

template <typename T>
void launch_sample(Ctrl* ctrl, const Table<T>* tbl, int nsub, long N, double* part, int nblk,
                   double* sample_t, double* sample_m, int cap, hipStream_t st, Prof* prof) {
  ProfScope ps(prof, P_REDUCE, st);
  hipLaunchKernelGGL((k_sample_part<T>), dim3(nblk), dim3(256), 0, st, ctrl, tbl, nsub, N, part);
  hipLaunchKernelGGL(k_sample_final, dim3(1), dim3(64), 0, st, ctrl, part, nblk, N, nsub, sample_t,
                     sample_m, cap);
}

__global__ void k_energy_final(const double* epart, int nblk, double* out) {
  const int t = threadIdx.x;
  if (t >= kNE) return;
  double acc = 0.0;
  for (int b = 0; b < nblk; ++b) acc += epart[(long)b * kNE + t];
  out[t] = acc;
}

void launch_energy_final(const double* epart, int nblk, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_energy_final, dim3(1), dim3(64), 0, st, epart, nblk, out);
}

#define INST(T)                                                                              \
  template void launch_field<T>(const FieldArgs<T>&, bool, hipStream_t, Prof*);             \
  template void launch_combine2<T>(const Table<T>*, const Ctrl*, long, int, hipStream_t,    \
                                   Prof*);                                                   \
  template void launch_control<T>(Ctrl*, Table<T>*, const double*, int, int, hipStream_t,   \
                                  Prof*);                                                    \
  template void launch_sample<T>(Ctrl*, const Table<T>*, int, long, double*, int, double*,  \
                                 double*, int, hipStream_t, Prof*);                          \
  template void launch_field_multi<T>(const FieldArgs<T>*, const int2*, int, int, int, int,   \
                                      hipStream_t);                                          \
  template void launch_step_multi<T>(const StepWork<T>*, int, long, hipStream_t);
INST(float)
INST(double)

}  // namespace mmp
