// Field/torque/RK kernels: argument structs and launchers.
#pragma once

#include "common.h"
#include "prof.h"

namespace mmp {

constexpr int kNE = 10;  // energy terms, order of MMP_NENERGY
constexpr int kTileX = 64, kTileY = 4;

template <typename T>
struct SubC {
  T ms;                       // Ms (demag source)
  T cex, cnn, ccell;          // 2A11/Ms, A12/Ms, 4A0/(Ms a^2)
  T cdmi, kdmi;               // 2D/Ms, ghost slope -D/(2 A11)
  T dh[3];                    // homogeneous DMI: -d/Ms1 (first), +d/Ms2 (second)
  T cku1, cku2, u[3];         // 2Ku1/Ms, 4Ku2/Ms, axis
  T ckc, c1[3], c2[3], c3[3]; // 2Kc1/Ms, cubic frame
  T cmel1, cmel2;             // 2B1/Ms, 2B2/Ms
  T gl, alpha;                // gamma/(1+alpha^2), alpha
  T zu[3], zla, zlb;          // drift velocity, (1+xi a)/(1+a^2), (xi-a)/(1+a^2)
  int has_zl;
  int nonzero;                // Ms != 0
  double Ms_d, Ku1_d, Ku2_d, Kc1_d, B1_d, B2_d;
};

template <typename T>
struct FieldArgs {
  int nx, ny, nz, nsub;
  long N;
  T dx, dy, dz, idx2, idy2, idz2, i2dx, i2dy, i2dz;
  SubC<T> sc[3];
  T bext[3];
  int dmi_layer;
  int has_demag, has_dmi, has_anis_u, has_anis_c, has_mel;
  int per_x, per_y;           // periodic axes: neighbours wrap, no DMI boundary
  int has_dmih;               // homogeneous inter-sublattice DMI
  // DMI tensors (Eq. 4) with the Neumann condition of Eq. 6 (gdmi != 0):
  // eW = W^(s) (rows: directions), eA = A11^(s), eA12 = A12 for the ghosts;
  // cW = -2 W^(s)/Ms^(s), cW12 = -2 W^(12)/Ms^(s) for the field
  int gdmi;
  T eW[2][3][3], eA[2], eA12;
  T cW[2][3][3], cW12[2][3][3];
  const uint16_t* grain;
  const T* gaxes;
  // grain boundaries (gbx != 0): A11 and A12 links between cells of
  // different grains scaled by gbx_scale
  int gbx;
  T gbx_scale;
  const T* Bd;
  const T* eps;
  const Table<T>* tbl;
  Ctrl* ctrl;
  int stage;
  int fuse2;
  double* errpart;
  uint32_t mask;
  T* bout;
  int out_torque;
  int add_zl;
  double* epart;
  double V;
  int nbx, nby, nb_pad;
  int zc, nzc;                // z planes per thread, z chunks (nzc * zc >= nz)
};

template <typename T>
void launch_field(const FieldArgs<T>& a, bool eval, hipStream_t st, Prof* prof);

// Per-grid pointers of a batch for the step controller and the stage-2
// combination (one entry per grid).
template <typename T>
struct StepWork {
  Ctrl* ctrl;
  Table<T>* tbl;
  const double* errpart;
  int nerr;
  int nsub;
  long N;
};

// Stage `stage` of many grids (no demag, no elasticity) in one launch:
// args[g] are the grids' field arguments in device memory, work[b] =
// (grid, block) for every field block of every grid.
template <typename T>
void launch_field_multi(const FieldArgs<T>* args, const int2* work, int nwork, int nsub, int stage,
                        int fuse2, hipStream_t st);
// step control of every grid, then its next stage-2 input
template <typename T>
void launch_step_multi(const StepWork<T>* w, int ngrids, long max_cells, hipStream_t st);

template <typename T>
void launch_combine2(const Table<T>* tbl, const Ctrl* ctrl, long Ncell, int nsub, hipStream_t st,
                     Prof* prof);

template <typename T>
void launch_control(Ctrl* ctrl, Table<T>* tbl, const double* errpart, int nerr, int elastic,
                    hipStream_t st, Prof* prof);

template <typename T>
void launch_sample(Ctrl* ctrl, const Table<T>* tbl, int nsub, long N, double* part, int nblk,
                   double* sample_t, double* sample_m, int cap, hipStream_t st, Prof* prof);

void launch_energy_final(const double* epart, int nblk, double* out, hipStream_t st);

}  // namespace mmp
