// Argument blocks and launchers of the power-of-two (register four-step)
// demag passes.
#pragma once

#include "common.h"

namespace mmp {

template <typename T>
struct X4Args {
  const Table<T>* tbl;
  const Ctrl* ctrl;
  int stage;
  T ms0, ms1;
  int nsub;
  cpx<T>* S1;
  T* Bd;
  const cpx<T>* tw4;
  int nx, ny, nz, Hx, ldy, ty;
};

template <typename T>
struct Y4Args {
  const Ctrl* ctrl;
  const cpx<T>* in;
  cpx<T>* out;
  const cpx<T>* tw4;
  int nlines, nvalid_in, ld_in, nvalid_out, ld_out, nl;
};

template <typename T>
struct M4Args {
  const Ctrl* ctrl;
  cpx<T>* S1;
  const T* K;
  const cpx<T>* tw4;
  int ny, Hx, Hy, ldy, nk;
};

template <typename T>
struct Z4Args {
  const Ctrl* ctrl;
  cpx<T>* S2;
  const T* K;
  int nz, Hx, Py, Hy, Hz, tk, nb_pad;
};

template <typename T>
void launch_y4(int L, bool inv, dim3 g, int thr, size_t lds, hipStream_t st, const Y4Args<T>& a);
template <typename T>
void launch_x4(int L, bool inv, dim3 g, int thr, size_t lds, hipStream_t st, const X4Args<T>& a);
template <typename T>
void launch_m4(int L, dim3 g, int thr, size_t lds, hipStream_t st, const M4Args<T>& a);
template <typename T>
void launch_z4(int PZ, dim3 g, int thr, size_t lds, hipStream_t st, const Z4Args<T>& a);

}  // namespace mmp
