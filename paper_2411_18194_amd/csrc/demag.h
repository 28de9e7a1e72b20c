// Demagnetising-field convolution on the GPU: plan, buffers, launchers.
#pragma once

#include <vector>

#include "common.h"
#include "fft_engine.h"
#include "prof.h"

namespace mmp {

// Geometry of the padded convolution.  Spectra are stored with the y axis
// contiguous:  S1[c][z][kx][y] (y < ny, line stride ldy)  after the x pass,
// S2[c][z][kx][ky] (ky < Py) after the forward y pass (3-D grids only).
// The kernel spectrum is real and stored on one octant:
// K[comp][kz <= Pz/2][kx < Hx][ky <= Py/2], comp = xx, yy, zz, xy, xz, yz.
//
// The pads and the launch shapes below are the tunable part of the plan;
// every valid choice computes the same convolution (the launch shapes only
// regroup identical per-line transforms, except zq, which changes the
// factorisation of the z transform).
struct DemagPlan {
  int nx = 0, ny = 0, nz = 0;
  int Px = 0, Py = 0, Pz = 0, Hx = 0, Hy = 0, Hz = 0;
  int ldy = 0;                      // multiple of 16, so any x block shape fits
  Rad rx{}, ry{}, rz{};
  // power-of-two axes use the register four-step kernels
  bool p2x = false, p2y = false, p2z = false;
  // launch shapes
  int tyf = 0, tyi = 0;             // x passes: rows (even, <= 16) per block, fwd / inv
  int nlyf = 0, nlyi = 0;           // y passes: lines per block, fwd / inv
  int nk = 0;                       // 2-D fused y pass: kx columns per block
  int tk = 0;                       // mixed-radix z pass: ky columns per block
  int zq = 1, zw = 1, zt = 0;       // register z pass: lanes per column, waves hint, threads
  int zmode = 0;                    // register z pass: 1 = kernel values staged through LDS
  // image repetitions per axis; > 0 makes the axis periodic (x and y only):
  // P = n, no zero padding, the kernel summed over the images
  int rep[3] = {0, 0, 0};
  // axes (bits 0/1/2 = x/y/z) forced onto the mixed-radix LDS kernels
  // although their pads are powers of two
  int force_lds = 0;
  size_t s1_elems = 0, s2_elems = 0, k_elems = 0;
};

// Plan with the default launch shapes for the given pads (nullptr: the
// smallest even 7-smooth pads, n on a periodic axis) and image repetitions
// rep (nullptr: open boundaries).  Returns 0, or -1 for an unsupported pad.
int demag_plan(int nx, int ny, int nz, int real_bytes, const int* pads, DemagPlan* p,
               const int* rep = nullptr);
// 0 if every launch shape of p is within the kernels' limits.
int demag_plan_check(const DemagPlan& p, int real_bytes);

enum DemagPass { DP_XF = 0, DP_YF, DP_Z, DP_YI, DP_XI, DP_M2, DP_COUNT };

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
// the array `src` directly.  M = Ms0 m0 + Ms1 m1 (+ Ms2 m2 for three
// sublattices).
template <typename T>
void demag_field(const DemagPlan& p, const DemagBufs<T>& b, const Table<T>* tbl, int stage,
                 const Ctrl* ctrl, T ms0, T ms1, int nsub, hipStream_t st, Prof* prof,
                 T ms2 = T(0));

// One pass of demag_field on its own (the autotuner times them one by one).
template <typename T>
void demag_pass(int pass, const DemagPlan& p, const DemagBufs<T>& b, const Table<T>* tbl,
                int stage, const Ctrl* ctrl, T ms0, T ms1, int nsub, hipStream_t st,
                T ms2 = T(0));

// Times the candidate launch shapes of every pass for the pads of *p on the
// buffers b and keeps the fastest in *p.  Returns the time of one demag
// evaluation with the chosen shapes in ms (< 0 on a HIP error).
template <typename T>
double demag_tune(DemagPlan* p, const DemagBufs<T>& b, const Table<T>* tbl, T ms0, T ms1,
                  int nsub, hipStream_t st, T ms2 = T(0));

// FP64 tensor on the non-negative offsets and its transformed octant
// spectrum.  n6 (6*N doubles, device) receives the tensor; kout the scaled
// spectrum (k_elems values of type T, device).
template <typename T>
int demag_kernel_build(const DemagPlan& p, double dx, double dy, double dz, double* n6,
                       T* kout, hipStream_t st);

// The tensor from every cell of the grid to a layer of cells centred at
// height zt (layer 0 of the grid centred at 0): 6*nz*(2ny-1)*(2nx-1)
// doubles [c][z][Y + ny - 1][X + nx - 1] (device).
int stray_kernel_build(int nx, int ny, int nz, double dx, double dy, double dz, double zt,
                       double* k6, hipStream_t st);
int demag_tensor_only(int nx, int ny, int nz, double dx, double dy, double dz, double* n6,
                      hipStream_t st);

// One grid of a batched demag evaluation: its plan (pads; its launch
// shapes are not used), buffers, state table, controller and moments.
template <typename T>
struct DemagMember {
  const DemagPlan* plan;
  DemagBufs<T> bufs;
  const Table<T>* tbl;
  const Ctrl* ctrl;
  T ms0, ms1, ms2;
  int nsub;
};

// The demag passes of many grids of any pads, each pass one launch for all
// of them over a device work table of (grid, block) entries, through the
// mixed-radix LDS kernels with 256-thread blocks.  A grid's field is bitwise
// the one its own plan gives with every axis on those kernels (force_lds =
// 7): the per-line arithmetic of the LDS kernels does not depend on how
// lines are grouped into blocks.
// Whether a grid with plan p can join a batched demag evaluation (its lines
// fit one 256-thread block of the LDS kernels).
bool demag_multi_fits(const DemagPlan& p);

template <typename T>
class DemagMulti {
 public:
  DemagMulti() = default;
  DemagMulti(const DemagMulti&) = delete;
  DemagMulti& operator=(const DemagMulti&) = delete;
  ~DemagMulti() { release(); }
  // device tables for the members (synchronous); 0, or MMP_E_NOMEM /
  // MMP_E_HIP
  int build(const std::vector<DemagMember<T>>& members, hipStream_t st);
  // B_d of every member for the stage input of `stage`
  void launch(int stage, hipStream_t st) const;
  bool empty() const { return impl == nullptr; }
  void release();

 private:
  struct Impl;
  Impl* impl = nullptr;
};

template <typename T>
void build_twiddles(cpx<T>* tw, int L, hipStream_t st);
template <typename T>
void build_twiddles4(cpx<T>* tw, int L, hipStream_t st);
int split_l2(int L);

}  // namespace mmp
