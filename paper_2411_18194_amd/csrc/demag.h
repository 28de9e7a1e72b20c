// Demagnetising-field convolution on the GPU: plan, buffers, launchers.
#pragma once

#include "common.h"
#include "fft_engine.h"
#include "prof.h"

namespace mmp {

// Geometry of the padded convolution.  Spectra are stored with the y axis
// contiguous:  S1[c][z][kx][y] (y < ny, line stride ldy)  after the x pass,
// S2[c][z][kx][ky] (ky < Py) after the forward y pass (3-D grids only).
// The kernel spectrum is real and stored on one octant:
// K[comp][kz <= Pz/2][kx < Hx][ky <= Py/2], comp = xx, yy, zz, xy, xz, yz.
struct DemagPlan {
  int nx = 0, ny = 0, nz = 0;
  int Px = 0, Py = 0, Pz = 0, Hx = 0, Hy = 0, Hz = 0;
  int ldy = 0;
  Rad rx{}, ry{}, rz{};
  // launch shapes
  int ty = 0, thr_x = 0;            // x passes: rows per block (even), threads
  int nly = 0, thr_y = 0;           // y passes: lines per block, threads
  int tk = 0, lsz = 0, thr_z = 0;   // z pass: ky per block, LDS line stride
  int nk2 = 0, thr_m2 = 0;          // 2-D fused y pass: kx columns per block
  // power-of-two axes use the register four-step kernels
  bool p2x = false, p2y = false, p2z = false;
  int nly4 = 0, nk4 = 0, tk4 = 0;
  size_t s1_elems = 0, s2_elems = 0, k_elems = 0;
};

int demag_plan(int nx, int ny, int nz, int real_bytes, DemagPlan* p);

template <typename T>
struct DemagBufs {
  cpx<T>* S1 = nullptr;
  cpx<T>* S2 = nullptr;
  T* K = nullptr;           // octant spectrum, scaled by -mu0/(Px Py Pz)
  cpx<T>* twx = nullptr;    // exp(-2 pi i j/P) tables
  cpx<T>* twy = nullptr;
  cpx<T>* twz = nullptr;
  cpx<T>* tw4x = nullptr;   // four-step tables [k1][t] = exp(-2 pi i t k1/L)
  cpx<T>* tw4y = nullptr;
  T* Bd = nullptr;          // output field [3][N]
};

// B_d for the stage input of `stage` (see stage_in) or, with stage == 0, for
// the array `src` directly.  M = Ms0 m0 + Ms1 m1.
template <typename T>
void demag_field(const DemagPlan& p, const DemagBufs<T>& b, const Table<T>* tbl, int stage,
                 const Ctrl* ctrl, T ms0, T ms1, int nsub, hipStream_t st, Prof* prof);

// FP64 tensor on the non-negative offsets and its transformed octant
// spectrum.  n6 (6*N doubles, device) receives the tensor; kout the scaled
// spectrum (k_elems values of type T, device).
template <typename T>
int demag_kernel_build(const DemagPlan& p, double dx, double dy, double dz, double* n6,
                       T* kout, hipStream_t st);

int demag_tensor_only(int nx, int ny, int nz, double dx, double dy, double dz, double* n6,
                      hipStream_t st);

template <typename T>
void build_twiddles(cpx<T>* tw, int L, hipStream_t st);
template <typename T>
void build_twiddles4(cpx<T>* tw, int L, hipStream_t st);
int split_l2(int L);

}  // namespace mmp
