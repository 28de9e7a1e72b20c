// Elastodynamics kernels (Eq. 7, 8): strain, stress with traction rows,
// divergence, magnetoelastic force, and the (u, v) Runge-Kutta stages.
#pragma once

#include "common.h"
#include "prof.h"

namespace mmp {

template <typename T>
struct ElasticArgs {
  int nx, ny, nz, nsub;
  long N;
  T dx, dy, dz;
  T C11, C12, C44, eta, inv_rho;
  double trac_amp, trac_omega;   // sigma_xz(t) = amp sin(omega t) on x = 0
  T B1[2], B2[2];
  int mel[2];                    // sublattice contributes a force
  const Table<T>* tbl;
  Ctrl* ctrl;
  int stage;                     // 1..7, or 0 = evaluate at (un, vn)
  int fuse2;
  T* eps;                        // [6][N] strain of the stage input
  T* epsv;                       // [6][N] strain rate (strain of v), beta != 0
  T beta;                        // Rayleigh stiffness coefficient, s
  T* sig;                        // [6][N] stress with traction rows
  double* epart;                 // [nblk] elastic energy partials (eval)
  double V;
  double rho;
};

// strain of the stage-s displacement into eps (consumed by the field
// kernel's magnetoelastic term and by the stress kernel)
template <typename T>
void launch_strain(const ElasticArgs<T>& a, hipStream_t st, Prof* prof);
// stress, divergence, forces, k_u/k_v and the next stage's u, v inputs
template <typename T>
void launch_elastic_stage(const ElasticArgs<T>& a, bool eval, hipStream_t st, Prof* prof);
template <typename T>
void launch_elastic_combine2(const Table<T>* tbl, const Ctrl* ctrl, long N, hipStream_t st,
                             Prof* prof);

}  // namespace mmp
