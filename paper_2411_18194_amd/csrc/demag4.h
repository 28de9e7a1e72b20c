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
  T ms0, ms1, ms2;
  int nsub;
  cpx<T>* S1;
  T* Bd;
  const cpx<T>* tw4;
  int nx, ny, nz, Hx, ldy, ty;
  int lnl;  // log2(ty / 2)
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

// Register z pass variants that are built: a lane holds the three
// components of PZ/zq points, data_vgprs 32-bit registers; variants that
// would hold more than 192 are not built, and a waves-per-SIMD hint zw > 1 is
// built only where zw times the data still fits the 512-register file with
// a quarter to spare.
constexpr int zreg_data_vgprs(int real_bytes, int pz, int zq) {
  return 3 * (pz / zq) * 2 * (real_bytes / 4);
}
constexpr bool zreg_ok(int real_bytes, int pz, int zq) {
  return (zq == 1 || zq == 2 || zq == 4) && pz >= 2 && pz <= 64 && (zq == 1 || pz / zq >= 2) &&
         zreg_data_vgprs(real_bytes, pz, zq) <= 192;
}
// LDS of one block of the register z pass with its kernel values staged
// through LDS (32-bit values only, one wave per SIMD): six rows of one word
// per lane for each of the PZ/2 + 1 mirrored planes (one lane per column) or
// PZ/zq registers (zq lanes per column).
constexpr long zk_lds_bytes(int pz, int zq, int threads) {
  return (long)(threads / 64) * 6 * (zq == 1 ? pz / 2 + 1 : pz / zq) * 64 * 4;
}
constexpr bool zreg_waves_ok(int real_bytes, int pz, int zq, int zw) {
  return zreg_ok(real_bytes, pz, zq) &&
         (zw == 1 || ((zw == 2 || zw == 4) && zreg_data_vgprs(real_bytes, pz, zq) * zw <= 384));
}

// full: the forward transform's input fills its whole length (a periodic
// axis); otherwise the upper half of a forward line is zero padding.
template <typename T>
void launch_y4(int L, bool inv, bool full, dim3 g, int thr, size_t lds, hipStream_t st,
               const Y4Args<T>& a);
// dynamic LDS bytes of a power-of-two x block of nl lines of L points
// (complex value bytes vb): the FP32 forward pass holds half a line per
// line from 64 points on (plus one aligned group of 32), the others a
// whole line
inline size_t x4_lds_bytes(int L, int nl, bool inv, int vb) {
  const long per = (!inv && L >= 64 && vb == 8) ? L / 2 + 32 : L;
  return (size_t)nl * (size_t)per * (size_t)vb;
}
template <typename T>
void launch_x4(int L, bool inv, bool full, dim3 g, int thr, size_t lds, hipStream_t st,
               const X4Args<T>& a);
template <typename T>
void launch_m4(int L, bool full, dim3 g, int thr, size_t lds, hipStream_t st,
               const M4Args<T>& a);
template <typename T>
void launch_z4(int PZ, int q, int w, int mode, dim3 g, int thr, hipStream_t st,
               const Z4Args<T>& a);

}  // namespace mmp
