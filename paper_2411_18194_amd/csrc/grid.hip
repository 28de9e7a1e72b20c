// Grid driver: device buffers, parameter coefficients, and the enqueueing
// of Dormand-Prince steps whose control lives on the device.
#include <algorithm>
#include <atomic>
#include <cstddef>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>

#include "grid.h"
#include "stray.h"

namespace mmp {

// the pair's stage count and index are written to the device table together
static_assert(offsetof(Table<float>, rk) == offsetof(Table<float>, ns) + sizeof(int), "");
static_assert(offsetof(Table<double>, rk) == offsetof(Table<double>, ns) + sizeof(int), "");

// Plans chosen by the autotuner, per (nx, ny, nz, real bytes, demag on,
// device); new grids of a tuned shape start from the tuned plan.
using PlanKey = std::tuple<int, int, int, int, int, int, int, int>;
struct TunedPlan {
  DemagPlan demag;
  double demag_ms;
  int field_zc;
  double field_ms;
};
static std::mutex g_plan_mu;
static std::map<PlanKey, TunedPlan> g_plans;

static int current_device() {
  int dev = 0;
  (void)hipGetDevice(&dev);
  return dev;
}

// ---------------------------------------------- device-pointer state I/O --
// The state buffers are found through the device pointer table, which the
// step controller swaps on the device: reading it there keeps these copies
// ordered on the grid's stream with no host round trip.
template <typename T>
__global__ void k_state_in(const Table<T>* tbl, const double* m, long nm, const double* u,
                           const double* v, long n3, int elastic) {
  const long stride = (long)gridDim.x * blockDim.x;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < nm; i += stride)
    tbl->yn[i] = (T)m[i];
  if (elastic)
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n3; i += stride) {
      tbl->un[i] = u ? (T)u[i] : T(0);
      tbl->vn[i] = v ? (T)v[i] : T(0);
    }
}

template <typename T>
__global__ void k_state_out(const Table<T>* tbl, const Ctrl* c, double* m, long nm, double* u,
                            double* v, long n3, int elastic, double* t_dt) {
  const long i0 = blockIdx.x * (long)blockDim.x + threadIdx.x;
  const long stride = (long)gridDim.x * blockDim.x;
  if (m)
    for (long i = i0; i < nm; i += stride) m[i] = (double)tbl->yn[i];
  for (long i = i0; i < n3; i += stride) {
    if (u) u[i] = elastic ? (double)tbl->un[i] : 0.0;
    if (v) v[i] = elastic ? (double)tbl->vn[i] : 0.0;
  }
  if (t_dt && i0 == 0) {
    t_dt[0] = c->t;
    t_dt[1] = c->dt;
  }
}

// a fresh controller at time t with first step dt (mmp_set_state's reset)
__global__ void k_ctrl_reset(Ctrl* c, double t, double dt) {
  Ctrl z{};
  z.t = t;
  z.dt = dt;
  *c = z;
}

template <typename T>
__global__ void k_widen(const T* in, double* out, long n) {
  const long stride = (long)gridDim.x * blockDim.x;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += stride)
    out[i] = (double)in[i];
}

static unsigned copy_blocks(long n) {
  const long b = (n + 255) / 256;
  return (unsigned)(b < 1 ? 1 : (b > 4096 ? 4096 : b));
}

// device memory of the stream's device (MMP_E_ARG otherwise)
static int check_device_buffer(const void* ptr, hipStream_t st, const char* what) {
  if (!ptr) return 0;
  hipPointerAttribute_t at{};
  if (hipPointerGetAttributes(&at, ptr) != hipSuccess || at.type != hipMemoryTypeDevice) {
    (void)hipGetLastError();
    set_error(std::string(what) + " is not device memory");
    return MMP_E_ARG;
  }
  int dev = 0;
  if (hipStreamGetDevice(st, &dev) != hipSuccess) {
    set_error("hipStreamGetDevice failed");
    return MMP_E_HIP;
  }
  if (at.device != dev) {
    set_error(std::string(what) + " is on another device than the grid");
    return MMP_E_ARG;
  }
  return 0;
}

template <typename T>
struct Buf {
  T* p = nullptr;
  size_t n = 0;
  int alloc(size_t count) {
    n = count;
    if (count == 0) return 0;
    DeviceLock lk(device_mutex());
    return hipMalloc(&p, count * sizeof(T)) == hipSuccess ? 0 : -1;
  }
  void release() {
    if (p) {
      DeviceLock lk(device_mutex());
      (void)hipFree(p);
    }
    p = nullptr;
    n = 0;
  }
};

template <typename T>
struct Grid final : GridBase {
  // state and stages
  Buf<T> y[2], sa, sb, k[7];
  Buf<T> u[2], v[2], usa, usb, vsa, vsb, ku[7], kv[7], eps, epsv, sig;
  Buf<T> Bd, gax;
  Buf<uint16_t> gid;
  Buf<double> errpart, epart, eout, spart, samp_t, samp_m, elpart;
  Buf<Table<T>> dtbl;
  Buf<Ctrl> dctrl;
  Buf<Ctrl> sctrl;        // controller of an on-demand average (summary)
  Buf<double> sres;       // its time and averages
  Ctrl* hctrl = nullptr;  // pinned mirror
  // demag
  DemagPlan plan{};
  DemagBufs<T> db{};
  Buf<cpx<T>> S1, S2, tw;
  Buf<T> K;
  bool demag_built = false;
  // layout of the current allocation
  bool allocated = false;
  int a_nsub = 0, a_elastic = 0, a_demag = 0, a_pbc[2] = {0, 0};
  bool k1_valid = false;
  double t_host = 0.0, dt_host = 0.0;
  FieldArgs<T> fa{};
  ElasticArgs<T> ea{};
  int nblk = 0, nb_pad = 0, nsamp_blk = 0;
  int samp_cap = 0;

  ~Grid() override {
    if (stream) (void)hipStreamSynchronize(stream);
    free_all();
    DeviceLock lk(device_mutex());
    if (hctrl) (void)hipHostFree(hctrl);
    for (int i = 0; i < 2; ++i) {
      if (chunk_ev[i]) (void)hipEventDestroy(chunk_ev[i]);
      if (chunk_ctrl[i]) (void)hipHostFree(chunk_ctrl[i]);
    }
  }

  void free_all() {
    drop_graphs();
    for (auto* b : {&y[0], &y[1], &sa, &sb, &u[0], &u[1], &v[0], &v[1], &usa, &usb, &vsa, &vsb,
                    &eps, &epsv, &sig, &Bd, &gax, &K, &evalb})
      b->release();
    for (int i = 0; i < 7; ++i) { k[i].release(); ku[i].release(); kv[i].release(); }
    gid.release();
    for (auto* b : {&errpart, &epart, &eout, &spart, &samp_t, &samp_m, &elpart}) b->release();
    dtbl.release();
    dctrl.release();
    sctrl.release();
    sres.release();
    S1.release(); S2.release(); tw.release();
    plan = DemagPlan{};
    allocated = false;
    demag_built = false;
  }

  long long bytes() const override {
    long long b = 0;
    auto add = [&](size_t n, size_t sz) { b += (long long)(n * sz); };
    add(y[0].n * 4 + 7 * k[0].n, sizeof(T));
    add((u[0].n * 4 + usa.n * 4 + 14 * ku[0].n + eps.n + sig.n), sizeof(T));
    add(Bd.n + K.n, sizeof(T));
    add(S1.n + S2.n + tw.n, sizeof(cpx<T>));
    return b;
  }

  int alloc_layout() {
    free_all();
    const int ns = p.nsub;
    const size_t nm = (size_t)ns * 3 * N;
    int rc = 0;
    rc |= y[0].alloc(nm); rc |= y[1].alloc(nm); rc |= sa.alloc(nm); rc |= sb.alloc(nm);
    for (int i = 0; i < 7; ++i) rc |= k[i].alloc(nm);
    if (p.elastic) {
      const size_t n3 = 3 * (size_t)N;
      rc |= u[0].alloc(n3); rc |= u[1].alloc(n3); rc |= v[0].alloc(n3); rc |= v[1].alloc(n3);
      rc |= usa.alloc(n3); rc |= usb.alloc(n3); rc |= vsa.alloc(n3); rc |= vsb.alloc(n3);
      for (int i = 0; i < 7; ++i) { rc |= ku[i].alloc(n3); rc |= kv[i].alloc(n3); }
      rc |= eps.alloc(6 * (size_t)N);
      rc |= epsv.alloc(6 * (size_t)N);
      rc |= sig.alloc(6 * (size_t)N);
    }
    // partial sums for the smallest z chunk (one plane per thread)
    const int nbx = (nx + kTileX - 1) / kTileX, nby = (ny + kTileY - 1) / kTileY;
    const int nb_max = round_up(nbx * nby * nz, 8);
    rc |= errpart.alloc(nb_max);
    rc |= epart.alloc((size_t)nb_max * kNE);
    rc |= eout.alloc(kNE);
    nsamp_blk = (int)std::min<long>(256, (N + 255) / 256);
    rc |= spart.alloc((size_t)nsamp_blk * 9);
    rc |= elpart.alloc((N + 255) / 256);
    rc |= dtbl.alloc(1);
    rc |= dctrl.alloc(1);
    bool cached = false;
    DemagPlan np;
    {
      std::lock_guard<std::mutex> lk(g_plan_mu);
      auto it = g_plans.find(plan_key());
      if (it != g_plans.end()) {
        np = it->second.demag;
        tuned_ms = it->second.demag_ms;
        field_zc = it->second.field_zc;
        field_ms = it->second.field_ms;
        cached = true;
      }
    }
    if (p.demag) {
      if (!cached && demag_plan(nx, ny, nz, (int)sizeof(T), nullptr, &np, p.pbc) != 0) {
        set_error("unsupported demag pads: each open axis pads to at most 4096, a periodic "
                  "axis needs n = 1 or n even and 7-smooth");
        free_all();
        return MMP_E_ARG;
      }
      rc |= Bd.alloc(3 * (size_t)N);
      db.Bd = Bd.p;
      if (!rc) rc |= install_plan(np);
    }
    if (rc) {
      set_error("device allocation failed");
      free_all();
      return MMP_E_NOMEM;
    }
    if (!hctrl) {
      DeviceLock lk(device_mutex());
      MMP_HIP_TRY(hipHostMalloc((void**)&hctrl, sizeof(Ctrl), 0));
    }
    // pointer table
    Table<T> t{};
    t.yn = y[0].p; t.ynew = y[1].p; t.sa = sa.p; t.sb = sb.p;
    for (int i = 0; i < 7; ++i) t.k[i] = k[i].p;
    if (p.elastic) {
      t.un = u[0].p; t.unew = u[1].p; t.vn = v[0].p; t.vnew = v[1].p;
      t.usa = usa.p; t.usb = usb.p; t.vsa = vsa.p; t.vsb = vsb.p;
      for (int i = 0; i < 7; ++i) { t.ku[i] = ku[i].p; t.kv[i] = kv[i].p; }
    }
    MMP_HIP_TRY(hipMemcpyAsync(dtbl.p, &t, sizeof(t), hipMemcpyHostToDevice, stream));
    MMP_HIP_TRY(hipMemsetAsync(y[0].p, 0, nm * sizeof(T), stream));
    if (p.elastic) {
      MMP_HIP_TRY(hipMemsetAsync(u[0].p, 0, 3 * N * sizeof(T), stream));
      MMP_HIP_TRY(hipMemsetAsync(v[0].p, 0, 3 * N * sizeof(T), stream));
    }
    Ctrl c{};
    MMP_HIP_TRY(hipMemcpyAsync(dctrl.p, &c, sizeof(c), hipMemcpyHostToDevice, stream));
    MMP_HIP_TRY(hipStreamSynchronize(stream));
    allocated = true;
    a_nsub = p.nsub; a_elastic = p.elastic; a_demag = p.demag;
    a_pbc[0] = p.pbc[0]; a_pbc[1] = p.pbc[1];
    state_set = false;
    return 0;
  }

  static void fill_sub(SubC<T>& s, const mmp_sublattice& b, const mmp_params& p) {
    const double Ms = b.Ms;
    const bool nz = Ms != 0.0;
    s.ms = (T)Ms;
    s.nonzero = nz ? 1 : 0;
    s.cex = (T)(nz ? 2.0 * b.A11 / Ms : 0.0);
    s.cnn = (T)(nz ? p.A12 / Ms : 0.0);
    s.ccell = (T)(nz ? 4.0 * p.A0 / (Ms * p.latcon * p.latcon) : 0.0);
    s.cdmi = (T)(nz ? 2.0 * b.Dint / Ms : 0.0);
    s.kdmi = (T)((b.A11 != 0.0 && b.Dint != 0.0) ? -b.Dint / (2.0 * b.A11) : 0.0);
    for (int c = 0; c < 3; ++c)
      s.dh[c] = (T)(nz && p.nsub == 2 ? (&b == &p.sub[0] ? -1.0 : 1.0) * p.dmi_homo[c] / Ms : 0.0);
    s.cku1 = (T)(nz ? 2.0 * b.Ku1 / Ms : 0.0);
    s.cku2 = (T)(nz ? 4.0 * b.Ku2 / Ms : 0.0);
    for (int c = 0; c < 3; ++c) s.u[c] = (T)b.anis_u[c];
    s.ckc = (T)(nz ? 2.0 * b.Kc1 / Ms : 0.0);
    const double* c1 = b.cub_c1;
    const double* c2 = b.cub_c2;
    const double c3[3] = {c1[1] * c2[2] - c1[2] * c2[1], c1[2] * c2[0] - c1[0] * c2[2],
                          c1[0] * c2[1] - c1[1] * c2[0]};
    for (int c = 0; c < 3; ++c) { s.c1[c] = (T)c1[c]; s.c2[c] = (T)c2[c]; s.c3[c] = (T)c3[c]; }
    s.cmel1 = (T)(nz ? 2.0 * b.B1 / Ms : 0.0);
    s.cmel2 = (T)(nz ? 2.0 * b.B2 / Ms : 0.0);
    const double al = b.alpha;
    s.gl = (T)(p.gamma / (1.0 + al * al));
    s.alpha = (T)al;
    double zu[3] = {0, 0, 0};
    if (nz)
      for (int c = 0; c < 3; ++c) zu[c] = b.zl_P * kMuB * p.j[c] / (kQe * Ms);
    s.has_zl = (zu[0] != 0.0 || zu[1] != 0.0 || zu[2] != 0.0) ? 1 : 0;
    for (int c = 0; c < 3; ++c) s.zu[c] = (T)zu[c];
    s.zla = (T)((1.0 + b.zl_xi * al) / (1.0 + al * al));
    s.zlb = (T)((b.zl_xi - al) / (1.0 + al * al));
    s.Ms_d = Ms; s.Ku1_d = b.Ku1; s.Ku2_d = b.Ku2; s.Kc1_d = b.Kc1; s.B1_d = b.B1; s.B2_d = b.B2;
  }

  // FFT buffers for plan np; a change of pads reallocates them and marks
  // the kernel spectrum for a rebuild.
  int install_plan(const DemagPlan& np) {
    drop_graphs();
    const bool same = S1.p && np.Px == plan.Px && np.Py == plan.Py && np.Pz == plan.Pz &&
                      np.s1_elems == plan.s1_elems && np.s2_elems == plan.s2_elems;
    if (!same) {
      if (stream) MMP_HIP_TRY(hipStreamSynchronize(stream));
      S1.release(); S2.release(); K.release(); tw.release();
      int rc = 0;
      rc |= S1.alloc(np.s1_elems);
      rc |= S2.alloc(np.s2_elems);
      rc |= K.alloc(np.k_elems);
      rc |= tw.alloc((size_t)2 * (np.Px + np.Py) + np.Pz);
      if (rc) {
        S1.release(); S2.release(); K.release(); tw.release();
        plan = DemagPlan{};
        set_error("device allocation failed");
        return MMP_E_NOMEM;
      }
      demag_built = false;
      k1_valid = false;
    }
    plan = np;
    set_demag_ptrs(db, S1.p, S2.p, K.p, tw.p, plan);
    return 0;
  }

  static void set_demag_ptrs(DemagBufs<T>& b, cpx<T>* s1, cpx<T>* s2, T* k, cpx<T>* t,
                             const DemagPlan& pl) {
    b.S1 = s1; b.S2 = s2; b.K = k;
    b.twx = t; b.twy = t + pl.Px; b.twz = t + pl.Px + pl.Py;
    b.tw4x = b.twz + pl.Pz; b.tw4y = b.tw4x + pl.Px;
  }

  void build_all_twiddles(const DemagBufs<T>& b, const DemagPlan& pl) {
    build_twiddles<T>(b.twx, pl.Px, stream);
    build_twiddles<T>(b.twy, pl.Py, stream);
    build_twiddles<T>(b.twz, pl.Pz, stream);
    build_twiddles4<T>(b.tw4x, pl.Px, stream);
    build_twiddles4<T>(b.tw4y, pl.Py, stream);
  }

  // twiddles and the transformed kernel for the current pads
  int build_demag() {
    DeviceLock lk(device_mutex());
    double* n6 = nullptr;
    MMP_HIP_TRY(hipMalloc(&n6, 6 * (size_t)N * sizeof(double)));
    build_all_twiddles(db, plan);
    const int rc = demag_kernel_build<T>(plan, d[0], d[1], d[2], n6, db.K, stream);
    (void)hipFree(n6);
    if (rc) {
      set_error("demag kernel build failed");
      return MMP_E_HIP;
    }
    demag_built = true;
    return 0;
  }

  // ------------------------------------------------------------- plan --
  double tuned_ms = 0.0, field_ms = 0.0;
  int field_zc = 0;  // z planes per field-kernel thread (0: not chosen yet)

  PlanKey plan_key() const {
    return PlanKey(nx, ny, nz, (int)sizeof(T), p.demag ? 1 : 0, current_device(), p.pbc[0],
                   p.pbc[1]);
  }

  // enough waves to cover the chip a few times over (8 per SIMD), with the
  // longest z march that still gives them: a small grid marches one plane
  // per thread, since its few blocks would otherwise leave most of the
  // chip idle while each thread walks its column
  int default_field_zc() const {
    const long waves = (long)((nx + kTileX - 1) / kTileX) * ((ny + kTileY - 1) / kTileY) * 4;
    int zc = nz;
    while (zc > 1 && waves * ((nz + zc - 1) / zc) < 8192) zc = (zc + 1) / 2;
    return zc;
  }

  void set_field_zc(int zc) {
    field_zc = std::max(1, std::min(zc, nz));
    fa.zc = field_zc;
    fa.nzc = (nz + field_zc - 1) / field_zc;
    nblk = fa.nbx * fa.nby * fa.nzc;
    nb_pad = round_up(nblk, 8);
    fa.nb_pad = nb_pad;
    drop_graphs();
  }

  int get_plan(mmp_plan* o) override {
    if (!params_set) {
      set_error("no plan: set parameters first");
      return MMP_E_STATE;
    }
    const uint32_t ss = o->struct_size;
    std::memset(o, 0, sizeof(*o));
    o->struct_size = ss;
    if (p.demag) {
      o->pad[0] = plan.Px; o->pad[1] = plan.Py; o->pad[2] = plan.Pz;
      o->x_rows[0] = plan.tyf; o->x_rows[1] = plan.tyi;
      o->y_lines[0] = plan.nlyf; o->y_lines[1] = plan.nlyi;
      o->xy_cols = plan.nk;
      o->z_cols = plan.tk;
      o->z_lanes = plan.zq; o->z_waves = plan.zw; o->z_threads = plan.zt;
      o->z_mode = plan.zmode;
      o->kinds = (plan.p2x ? 1u : 0u) | (plan.p2y ? 2u : 0u) | (plan.p2z ? 4u : 0u);
      o->lds_axes = plan.force_lds;
      o->demag_ms = tuned_ms;
    }
    o->field_zplanes = field_zc;
    o->field_ms = field_ms;
    return 0;
  }

  int set_plan(const mmp_plan* in) override {
    if (!params_set) {
      set_error("no plan: set parameters first");
      return MMP_E_STATE;
    }
    if (in->field_zplanes < 1 || in->field_zplanes > nz) {
      set_error("field_zplanes must be in 1..nz");
      return MMP_E_ARG;
    }
    if (p.demag) {
      DemagPlan np;
      if (demag_plan(nx, ny, nz, (int)sizeof(T), in->pad, &np, p.pbc) != 0) {
        set_error("unsupported pads: each must be 1 for a single cell, else even, 7-smooth, "
                  ">= 2n-1 and <= 4096");
        return MMP_E_ARG;
      }
      if (in->lds_axes < 0 || in->lds_axes > 7) {
        set_error("lds_axes: bits 0..2 only");
        return MMP_E_ARG;
      }
      np.force_lds = in->lds_axes;
      if (np.force_lds & 1) np.p2x = false;
      if (np.force_lds & 2) np.p2y = false;
      if (np.force_lds & 4) np.p2z = false;
      np.tyf = in->x_rows[0]; np.tyi = in->x_rows[1];
      np.nlyf = in->y_lines[0]; np.nlyi = in->y_lines[1];
      np.nk = in->xy_cols;
      np.tk = in->z_cols;
      if (np.p2z) {
        np.zq = in->z_lanes; np.zw = in->z_waves; np.zt = in->z_threads; np.zmode = in->z_mode;
      }
      if (demag_plan_check(np, (int)sizeof(T)) != 0) {
        set_error("plan launch shape outside the kernels' limits");
        return MMP_E_ARG;
      }
      int rc = install_plan(np);
      if (!rc && !demag_built) rc = build_demag();
      if (rc) return rc;
      tuned_ms = 0.0;
    }
    if (in->field_zplanes != field_zc) field_ms = 0.0;
    set_field_zc(in->field_zplanes);
    return 0;
  }

  // mean time of one field-kernel stage (stage 2 on scratch buffers, with a
  // controller of its own so a finished run does not skip the launches)
  double time_field(int zc, Ctrl* tctrl, int reps) {
    set_field_zc(zc);
    FieldArgs<T> a = fa;
    a.stage = 2;
    a.fuse2 = 0;
    a.ctrl = tctrl;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return -1.0;
    if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); return -1.0; }
    double ms = -1.0;
    launch_field<T>(a, false, stream, nullptr);
    if (hipEventRecord(e0, stream) == hipSuccess) {
      for (int r = 0; r < reps; ++r) launch_field<T>(a, false, stream, nullptr);
      float f = 0.f;
      if (hipGetLastError() == hipSuccess && hipEventRecord(e1, stream) == hipSuccess &&
          hipEventSynchronize(e1) == hipSuccess && hipEventElapsedTime(&f, e0, e1) == hipSuccess)
        ms = (double)f / reps;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return ms;
  }

  int tune_field() {
    Buf<Ctrl> tc;
    if (tc.alloc(1)) { set_error("device allocation failed"); return MMP_E_NOMEM; }
    Ctrl c{};
    c.h = 1e-15;
    MMP_HIP_TRY(hipMemcpy(tc.p, &c, sizeof(c), hipMemcpyHostToDevice));
    const int reps = N >= (1L << 22) ? 5 : N >= (1L << 16) ? 20 : 50;
    int best = field_zc;
    double bt = -1.0;
    for (int zc = 1;; zc *= 2) {
      const int z = std::min(zc, nz);
      const double t = time_field(z, tc.p, reps);
      if (t > 0.0 && (bt < 0.0 || t < bt)) { bt = t; best = z; }
      if (z == nz) break;
    }
    set_field_zc(best);
    field_ms = bt > 0.0 ? bt : 0.0;
    return 0;
  }

  int autotune(mmp_plan* out) override {
    if (!params_set) {
      set_error("autotune needs parameters");
      return MMP_E_STATE;
    }
    if (p.demag) {
      const int rc = tune_demag();
      if (rc) return rc;
    }
    MMP_HIP_TRY(hipStreamSynchronize(stream));
    if (int rc = tune_field()) return rc;
    {
      std::lock_guard<std::mutex> lk(g_plan_mu);
      g_plans[plan_key()] = {plan, tuned_ms, field_zc, field_ms};
    }
    return out ? get_plan(out) : 0;
  }

  int tune_demag() {
    auto pads_for = [](int n, int* c) {
      int k = 0;
      c[k++] = smooth_pad(n);
      if (n > 1) {
        int q = 1;
        while (q < 2 * n - 1) q *= 2;
        if (q != c[0] && q <= 4096) c[k++] = q;
      }
      return k;
    };
    int cx[2], cy[2], cz[2];
    int nxc = pads_for(nx, cx), nyc = pads_for(ny, cy);
    const int nzc = pads_for(nz, cz);
    // a periodic axis has the one cyclic length n
    if (p.pbc[0] > 0) { cx[0] = nx; nxc = 1; }
    if (p.pbc[1] > 0) { cy[0] = ny; nyc = 1; }
    const T ms0 = (T)p.sub[0].Ms, ms1 = ms_of(1), ms2 = ms_of(2);
    MMP_HIP_TRY(hipStreamSynchronize(stream));
    DemagPlan best{};
    double best_ms = -1.0;
    for (int i = 0; i < nxc; ++i)
      for (int j = 0; j < nyc; ++j)
        for (int k = 0; k < nzc; ++k) {
          const int pads[3] = {cx[i], cy[j], cz[k]};
          DemagPlan c;
          if (demag_plan(nx, ny, nz, (int)sizeof(T), pads, &c, p.pbc) != 0) continue;
          const bool cur = c.Px == plan.Px && c.Py == plan.Py && c.Pz == plan.Pz;
          DemagBufs<T> tb = db;
          Buf<cpx<T>> s1, s2, twb;
          Buf<T> kb;
          if (cur) {
            c.tyf = plan.tyf; c.tyi = plan.tyi; c.nlyf = plan.nlyf; c.nlyi = plan.nlyi;
            c.nk = plan.nk; c.tk = plan.tk;
            if (c.p2z == plan.p2z) { c.zq = plan.zq; c.zw = plan.zw; c.zt = plan.zt; }
            if (demag_plan_check(c, (int)sizeof(T)) != 0) c = plan;
          } else {
            if (s1.alloc(c.s1_elems) || s2.alloc(c.s2_elems) || kb.alloc(c.k_elems) ||
                twb.alloc((size_t)2 * (c.Px + c.Py) + c.Pz)) {
              s1.release(); s2.release(); kb.release(); twb.release();
              continue;  // this pad set does not fit next to the grid
            }
            set_demag_ptrs(tb, s1.p, s2.p, kb.p, twb.p, c);
            MMP_HIP_TRY(hipMemsetAsync(kb.p, 0, c.k_elems * sizeof(T), stream));
            build_all_twiddles(tb, c);
          }
          const double ms = demag_tune<T>(&c, tb, dtbl.p, ms0, ms1, p.nsub, stream, ms2);
          const hipError_t e = hipStreamSynchronize(stream);
          s1.release(); s2.release(); kb.release(); twb.release();
          if (e != hipSuccess) {
            set_error(std::string("autotune: ") + hipGetErrorString(e));
            return MMP_E_HIP;
          }
          if (ms > 0.0 && (best_ms < 0.0 || ms < best_ms)) {
            best_ms = ms;
            best = c;
          }
        }
    if (best_ms < 0.0) {
      set_error("autotune: no candidate plan could be timed");
      return MMP_E_HIP;
    }
    int rc = install_plan(best);
    if (!rc && !demag_built) rc = build_demag();
    if (rc) return rc;
    tuned_ms = best_ms;
    return 0;
  }

  // Ms of sublattice s, 0 past the grid's sublattices
  T ms_of(int s) const { return (T)(s < p.nsub ? p.sub[s].Ms : 0.0); }

  int apply_params() override {
    if (p.nsub >= 2)
      for (int s = 0; s < p.nsub; ++s)
        if (p.sub[s].Dint != 0.0) {
          set_error("interfacial DMI is implemented for one sublattice");
          return MMP_E_ARG;
        }
    if (!allocated || a_nsub != p.nsub || a_elastic != (p.elastic != 0) ||
        a_demag != (p.demag != 0) || a_pbc[0] != p.pbc[0] || a_pbc[1] != p.pbc[1]) {
      p.elastic = p.elastic != 0;
      p.demag = p.demag != 0;
      const int rc = alloc_layout();
      if (rc) return rc;
    }
    // grains
    gid.release();
    gax.release();
    if (p.ngrains > 0) {
      if (gid.alloc(N) || gax.alloc(3 * (size_t)p.ngrains)) {
        set_error("device allocation failed");
        return MMP_E_NOMEM;
      }
      MMP_HIP_TRY(hipMemcpy(gid.p, grain.data(), N * sizeof(uint16_t), hipMemcpyHostToDevice));
      std::vector<T> ax(grain_axes.begin(), grain_axes.end());
      MMP_HIP_TRY(hipMemcpy(gax.p, ax.data(), ax.size() * sizeof(T), hipMemcpyHostToDevice));
    }
    // demag kernel
    if (p.demag && !demag_built) {
      const int rc = build_demag();
      if (rc) return rc;
    }
    // field kernel arguments
    FieldArgs<T> a{};
    a.nx = nx; a.ny = ny; a.nz = nz; a.nsub = p.nsub; a.N = N;
    a.dx = (T)d[0]; a.dy = (T)d[1]; a.dz = (T)d[2];
    a.idx2 = (T)(1.0 / (d[0] * d[0])); a.idy2 = (T)(1.0 / (d[1] * d[1]));
    a.idz2 = (T)(1.0 / (d[2] * d[2]));
    a.i2dx = (T)(0.5 / d[0]); a.i2dy = (T)(0.5 / d[1]); a.i2dz = (T)(0.5 / d[2]);
    for (int s = 0; s < p.nsub; ++s) fill_sub(a.sc[s], p.sub[s], p);
    for (int c = 0; c < 3; ++c) a.bext[c] = (T)p.B_ext[c];
    a.dmi_layer = p.dmi_layer;
    a.has_demag = p.demag ? 1 : 0;
    a.has_dmi = (p.nsub == 1 && p.sub[0].Dint != 0.0) ? 1 : 0;
    a.has_anis_u = 0;
    a.has_anis_c = 0;
    a.has_mel = 0;
    for (int s = 0; s < p.nsub; ++s) {
      if (p.sub[s].Ku1 != 0.0 || p.sub[s].Ku2 != 0.0) a.has_anis_u = 1;
      if (p.sub[s].Kc1 != 0.0) a.has_anis_c = 1;
      if (p.elastic && (p.sub[s].B1 != 0.0 || p.sub[s].B2 != 0.0)) a.has_mel = 1;
    }
    a.grain = p.ngrains > 0 ? gid.p : nullptr;
    a.gaxes = p.ngrains > 0 ? gax.p : nullptr;
    a.Bd = Bd.p;
    a.eps = eps.p;
    a.tbl = dtbl.p;
    a.ctrl = dctrl.p;
    a.errpart = errpart.p;
    a.V = d[0] * d[1] * d[2];
    a.nbx = (nx + kTileX - 1) / kTileX;
    a.nby = (ny + kTileY - 1) / kTileY;
    a.has_dmih = (p.nsub == 2 && (p.dmi_homo[0] != 0.0 || p.dmi_homo[1] != 0.0 ||
                                  p.dmi_homo[2] != 0.0)) ? 1 : 0;
    a.gdmi = p.bc_eq6 ? 1 : 0;
    a.gbx = (p.ngrains > 0 && p.grain_exch_reduction != 0.0) ? 1 : 0;
    a.gbx_scale = (T)(1.0 - p.grain_exch_reduction);
    a.eA12 = (T)(p.nsub == 2 ? p.A12 : 0.0);
    for (int s = 0; s < 2; ++s) {
      const bool on = s < p.nsub;
      const double Ms = on ? p.sub[s].Ms : 0.0;
      a.eA[s] = (T)(on ? p.sub[s].A11 : 0.0);
      for (int i = 0; i < 3; ++i)
        for (int c = 0; c < 3; ++c) {
          a.eW[s][i][c] = (T)(on ? p.dmi_W[s][i][c] : 0.0);
          a.cW[s][i][c] = (T)(on && Ms != 0.0 ? -2.0 * p.dmi_W[s][i][c] / Ms : 0.0);
          a.cW12[s][i][c] =
              (T)(on && Ms != 0.0 && p.nsub == 2 ? -2.0 * p.dmi_W12[i][c] / Ms : 0.0);
        }
    }
    a.per_x = p.pbc[0] > 0 ? 1 : 0;
    a.per_y = p.pbc[1] > 0 ? 1 : 0;
    fa = a;
    set_field_zc(field_zc > 0 ? field_zc : default_field_zc());
    // the pair in use: its stage count and index, read by every stage kernel
    {
      const int v[2] = {RK::t[p.solver].ns, p.solver};
      MMP_HIP_TRY(hipMemcpy(reinterpret_cast<char*>(dtbl.p) + offsetof(Table<T>, ns), v,
                            sizeof(v), hipMemcpyHostToDevice));
    }
    // elastic arguments
    ElasticArgs<T> e{};
    e.nx = nx; e.ny = ny; e.nz = nz; e.nsub = p.nsub; e.N = N;
    e.dx = (T)d[0]; e.dy = (T)d[1]; e.dz = (T)d[2];
    e.C11 = (T)p.C11; e.C12 = (T)p.C12; e.C44 = (T)p.C44; e.eta = (T)p.eta;
    e.inv_rho = (T)(p.rho != 0.0 ? 1.0 / p.rho : 0.0);
    e.trac_amp = p.trac_amp;
    e.trac_omega = 2.0 * kPi * p.trac_freq;
    for (int s = 0; s < p.nsub; ++s) {
      e.B1[s] = (T)p.sub[s].B1;
      e.B2[s] = (T)p.sub[s].B2;
      e.mel[s] = (p.sub[s].Ms != 0.0 && (p.sub[s].B1 != 0.0 || p.sub[s].B2 != 0.0)) ? 1 : 0;
    }
    e.tbl = dtbl.p; e.ctrl = dctrl.p; e.eps = eps.p; e.sig = sig.p; e.epart = elpart.p;
    e.epsv = epsv.p; e.beta = (T)p.rayleigh;
    e.V = a.V; e.rho = p.rho;
    ea = e;
    drop_graphs();
    k1_valid = false;
    params_set = true;
    return 0;
  }

  int set_state(const double* m, const double* uu, const double* vv, double t) override {
    // work enqueued without a host synchronisation (mmp_step with a fixed
    // dt, mmp_run_fixed) may still swap the pointer table or write the
    // state and controller: let it finish before they are replaced
    MMP_HIP_TRY(hipStreamSynchronize(stream));
    const size_t nm = (size_t)p.nsub * 3 * N;
    // the pointer table may have been swapped by earlier steps: reset it
    Table<T> tb{};
    MMP_HIP_TRY(hipMemcpy(&tb, dtbl.p, sizeof(tb), hipMemcpyDeviceToHost));
    std::vector<T> tmp(nm);
    for (size_t i = 0; i < nm; ++i) tmp[i] = (T)m[i];
    MMP_HIP_TRY(hipMemcpy(tb.yn, tmp.data(), nm * sizeof(T), hipMemcpyHostToDevice));
    if (p.elastic) {
      std::vector<T> t3(3 * (size_t)N);
      for (size_t i = 0; i < t3.size(); ++i) t3[i] = uu ? (T)uu[i] : T(0);
      MMP_HIP_TRY(hipMemcpy(tb.un, t3.data(), t3.size() * sizeof(T), hipMemcpyHostToDevice));
      for (size_t i = 0; i < t3.size(); ++i) t3[i] = vv ? (T)vv[i] : T(0);
      MMP_HIP_TRY(hipMemcpy(tb.vn, t3.data(), t3.size() * sizeof(T), hipMemcpyHostToDevice));
    }
    Ctrl c{};
    c.t = t;
    c.dt = p.dt0 > 0 ? p.dt0 : 1e-14;
    MMP_HIP_TRY(hipMemcpy(dctrl.p, &c, sizeof(c), hipMemcpyHostToDevice));
    t_host = t;
    dt_host = c.dt;
    k1_valid = false;
    state_set = true;
    return 0;
  }

  int set_state_device(const double* m, const double* uu, const double* vv, double t) override {
    if (int rc = check_device_buffer(m, stream, "m")) return rc;
    if (int rc = check_device_buffer(uu, stream, "u")) return rc;
    if (int rc = check_device_buffer(vv, stream, "v")) return rc;
    const long nm = (long)p.nsub * 3 * N, n3 = 3L * N;
    const double dt = p.dt0 > 0 ? p.dt0 : 1e-14;
    hipLaunchKernelGGL(k_state_in<T>, dim3(copy_blocks(nm)), dim3(256), 0, stream, dtbl.p, m, nm,
                       uu, vv, n3, p.elastic ? 1 : 0);
    hipLaunchKernelGGL(k_ctrl_reset, dim3(1), dim3(1), 0, stream, dctrl.p, t, dt);
    MMP_HIP_TRY(hipGetLastError());
    t_host = t;
    dt_host = dt;
    k1_valid = false;
    state_set = true;
    return 0;
  }

  int get_state_device(double* m, double* uu, double* vv, double* t_dt) override {
    if (int rc = check_device_buffer(m, stream, "m")) return rc;
    if (int rc = check_device_buffer(uu, stream, "u")) return rc;
    if (int rc = check_device_buffer(vv, stream, "v")) return rc;
    if (int rc = check_device_buffer(t_dt, stream, "t_dt")) return rc;
    const long nm = (long)p.nsub * 3 * N, n3 = 3L * N;
    hipLaunchKernelGGL(k_state_out<T>, dim3(copy_blocks(nm)), dim3(256), 0, stream, dtbl.p,
                       dctrl.p, m, nm, uu, vv, n3, p.elastic ? 1 : 0, t_dt);
    MMP_HIP_TRY(hipGetLastError());
    return 0;
  }

  int get_state(double* m, double* uu, double* vv, double* t, double* dt) override {
    MMP_HIP_TRY(hipStreamSynchronize(stream));
    Table<T> tb{};
    MMP_HIP_TRY(hipMemcpy(&tb, dtbl.p, sizeof(tb), hipMemcpyDeviceToHost));
    Ctrl c{};
    MMP_HIP_TRY(hipMemcpy(&c, dctrl.p, sizeof(c), hipMemcpyDeviceToHost));
    if (m) {
      const size_t nm = (size_t)p.nsub * 3 * N;
      std::vector<T> tmp(nm);
      MMP_HIP_TRY(hipMemcpy(tmp.data(), tb.yn, nm * sizeof(T), hipMemcpyDeviceToHost));
      for (size_t i = 0; i < nm; ++i) m[i] = (double)tmp[i];
    }
    if (p.elastic && (uu || vv)) {
      std::vector<T> t3(3 * (size_t)N);
      if (uu) {
        MMP_HIP_TRY(hipMemcpy(t3.data(), tb.un, t3.size() * sizeof(T), hipMemcpyDeviceToHost));
        for (size_t i = 0; i < t3.size(); ++i) uu[i] = (double)t3[i];
      }
      if (vv) {
        MMP_HIP_TRY(hipMemcpy(t3.data(), tb.vn, t3.size() * sizeof(T), hipMemcpyDeviceToHost));
        for (size_t i = 0; i < t3.size(); ++i) vv[i] = (double)t3[i];
      }
    } else if (!p.elastic) {
      if (uu) std::fill(uu, uu + 3 * N, 0.0);
      if (vv) std::fill(vv, vv + 3 * N, 0.0);
    }
    if (t) *t = c.t;
    if (dt) *dt = c.dt;
    return 0;
  }

  // ---------------------------------------------------------- stages --
  void stage(int s, bool fuse2) {
    if (p.elastic) {
      ElasticArgs<T> e = ea;
      e.stage = s;
      launch_strain(e, stream, &prof);
    }
    if (p.demag)
      demag_field<T>(plan, db, dtbl.p, s, dctrl.p, (T)p.sub[0].Ms, ms_of(1), p.nsub, stream,
                     &prof, ms_of(2));
    FieldArgs<T> a = fa;
    a.stage = s;
    a.fuse2 = fuse2 ? 1 : 0;
    launch_field<T>(a, false, stream, &prof);
    if (p.elastic) {
      ElasticArgs<T> e = ea;
      e.stage = s;
      e.fuse2 = fuse2 ? 1 : 0;
      launch_elastic_stage<T>(e, false, stream, &prof);
    }
  }

  void combine2() {
    launch_combine2<T>(dtbl.p, dctrl.p, N, p.nsub, stream, &prof);
    if (p.elastic) launch_elastic_combine2<T>(dtbl.p, dctrl.p, N, stream, &prof);
  }

  // one attempt: stages 2..ns + control (+ sampling, + next stage-2 input)
  void attempt(bool fixed_mode, bool sampling) {
    const int ns = RK::t[p.solver].ns;
    for (int s = 2; s <= ns; ++s) stage(s, fixed_mode && s == ns);
    launch_control<T>(dctrl.p, dtbl.p, errpart.p, nblk, p.elastic ? 1 : 0, stream, &prof);
    if (sampling)
      launch_sample<T>(dctrl.p, dtbl.p, p.nsub, N, spart.p, nsamp_blk, samp_t.p, samp_m.p,
                       samp_cap, stream, &prof);
    if (!fixed_mode) combine2();
  }

  // ----------------------------------------------------------- graphs --
  // kGraphAttempts attempts captured once per kind (fixed, adaptive,
  // adaptive with sampling) and replayed; every kernel reads the step
  // controller and the buffer table on the device, so a replay needs no
  // new arguments.  Rebuilt whenever a kernel argument changes.
  static constexpr int kGraphAttempts = 8;
  hipGraphExec_t gexec[3] = {nullptr, nullptr, nullptr};
  bool graphs_on = true;

  void drop_graphs() {
    for (auto& e : gexec)
      if (e) {
        (void)hipGraphExecDestroy(e);
        e = nullptr;
      }
  }

  // graphs need a capturable stream and stay out of the way of profiling
  bool graphs_usable() const { return graphs_on && stream != nullptr && !prof.on; }

  int graph_for(int kind, hipGraphExec_t* out) {
    if (!gexec[kind]) {
      DeviceLock lk(device_mutex());
      hipGraph_t g = nullptr;
      MMP_HIP_TRY(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
      for (int i = 0; i < kGraphAttempts; ++i) attempt(kind == 0, kind == 2);
      const hipError_t e = hipStreamEndCapture(stream, &g);
      if (e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        set_error(std::string("graph capture: ") + hipGetErrorString(e));
        return MMP_E_HIP;
      }
      const hipError_t e2 = hipGraphInstantiate(&gexec[kind], g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (e2 != hipSuccess) {
        gexec[kind] = nullptr;
        set_error(std::string("graph instantiate: ") + hipGetErrorString(e2));
        return MMP_E_HIP;
      }
    }
    *out = gexec[kind];
    return 0;
  }

  // n attempts: whole graphs of kGraphAttempts, the rest launched directly
  int enqueue_attempts(bool fixed_mode, bool sampling, long long n) {
    long long left = n;
    if (graphs_usable() && n >= kGraphAttempts) {
      hipGraphExec_t ge = nullptr;
      const int kind = fixed_mode ? 0 : (sampling ? 2 : 1);
      int rc = graph_for(kind, &ge);
      if (rc) return rc;
      for (; left >= kGraphAttempts; left -= kGraphAttempts)
        MMP_HIP_TRY(hipGraphLaunch(ge, stream));
    }
    for (; left > 0; --left) attempt(fixed_mode, sampling);
    MMP_HIP_TRY(hipGetLastError());
    return 0;
  }

  int set_graphs(bool on) override {
    graphs_on = on;
    if (!on) drop_graphs();
    return 0;
  }

  int ensure_ready() {
    if (!params_set) { set_error("mmp_set_params has not been called"); return MMP_E_STATE; }
    if (!state_set) { set_error("mmp_set_state has not been called"); return MMP_E_STATE; }
    return 0;
  }

  // set up the controller for a run segment; returns after the first
  // stage-2 input is prepared
  int begin_segment(const Ctrl& init) {
    Ctrl c{};
    MMP_HIP_TRY(hipMemcpyAsync(hctrl, dctrl.p, sizeof(Ctrl), hipMemcpyDeviceToHost, stream));
    MMP_HIP_TRY(hipStreamSynchronize(stream));
    c = *hctrl;
    c.t_end = init.t_end; c.t_next = init.t_next; c.sample_every = init.sample_every;
    c.t0 = c.t; c.tol = init.tol; c.dt_min = init.dt_min; c.fixed = init.fixed;
    c.max_attempts = init.max_attempts;
    c.safety = p.safety > 0 ? p.safety : 0.8;
    c.fac_min = p.fac_min > 0 ? p.fac_min : 0.1;
    c.fac_max = p.fac_max > 0 ? p.fac_max : 2.0;
    c.dt_max = p.dt_max > 0 ? p.dt_max : 0.0;
    c.done = 0; c.status = 0; c.sample_k = init.fixed ? 0 : 1; c.nsamples = 0;
    c.sample_pending = 0; c.nonfinite = 0;
    if (init.fixed) {
      c.h = init.h;
      c.land = 0;
    } else {
      if (c.dt <= 0) c.dt = p.dt0 > 0 ? p.dt0 : 1e-14;
      if (c.dt_max > 0.0) c.dt = std::min(c.dt, c.dt_max);
      const double target = std::min(c.t_next, c.t_end);
      const double rem = target - c.t;
      c.land = c.dt >= rem ? 1 : 0;
      c.h = c.land ? rem : c.dt;
    }
    *hctrl = c;
    MMP_HIP_TRY(hipMemcpyAsync(dctrl.p, hctrl, sizeof(Ctrl), hipMemcpyHostToDevice, stream));
    if (!k1_valid) {
      stage(1, false);
      k1_valid = true;
    } else {
      combine2();
    }
    return 0;
  }

  int read_ctrl(Ctrl* c) {
    MMP_HIP_TRY(hipMemcpyAsync(hctrl, dctrl.p, sizeof(Ctrl), hipMemcpyDeviceToHost, stream));
    MMP_HIP_TRY(hipStreamSynchronize(stream));
    *c = *hctrl;
    return 0;
  }

  int run_fixed(double dt, long long n, mmp_step_info* info) override {
    int rc = ensure_ready();
    if (rc) return rc;
    if (!(dt > 0.0) || n < 0) { set_error("dt must be > 0 and nsteps >= 0"); return MMP_E_ARG; }
    if (n == 0) return 0;
    Ctrl init{};
    init.fixed = 1; init.h = dt; init.t_end = 1e300; init.t_next = 1e300;
    init.max_attempts = n; init.tol = 0; init.dt_min = 0;
    if ((rc = begin_segment(init))) return rc;
    if ((rc = enqueue_attempts(true, false, n))) return rc;
    if (info) {
      Ctrl c{};
      if ((rc = read_ctrl(&c))) return rc;
      info->t = c.t; info->dt = dt; info->err = 0; info->steps = c.steps; info->rejects = c.rejects;
      if (c.status) { set_error("non-finite state"); return c.status; }
    }
    return 0;
  }

  int step(double dt_fixed, mmp_step_info* info) override {
    if (dt_fixed > 0.0) return run_fixed(dt_fixed, 1, info);
    int rc = ensure_ready();
    if (rc) return rc;
    // adaptive: attempts until one is accepted
    Ctrl init{};
    init.fixed = 0; init.t_end = 1e300; init.t_next = 1e300;
    init.tol = p.tol > 0 ? p.tol : 1e-5;
    init.dt_min = p.dt_min > 0 ? p.dt_min : 1e-20;
    if ((rc = begin_segment(init))) return rc;
    Ctrl c{};
    const int64_t s0 = hctrl->steps;
    constexpr int kMaxAttempts = 1000;
    for (int it = 0; it < kMaxAttempts; ++it) {
      attempt(false, false);
      if ((rc = read_ctrl(&c))) return rc;
      if (c.status) { set_error(c.status == MMP_E_DT_UNDERFLOW ? "time step underflow" : "non-finite state"); return c.status; }
      if (c.steps > s0) break;
    }
    if (c.steps == s0) {
      set_error("adaptive step: no attempt accepted in 1000 tries");
      return MMP_E_STATE;
    }
    if (info) {
      info->t = c.t; info->dt = c.dt; info->err = c.err; info->steps = c.steps; info->rejects = c.rejects;
    }
    return 0;
  }

  int run(double t_end, const mmp_run_opts* o, mmp_run_info* info) override {
    int rc = ensure_ready();
    if (rc) return rc;
    Ctrl cur{};
    if ((rc = read_ctrl(&cur))) return rc;
    if (!(t_end > cur.t)) {
      if (info) { std::memset(info, 0, sizeof(*info)); info->t = cur.t; info->dt = cur.dt; }
      return 0;
    }
    const double every = o ? o->sample_every : 0.0;
    const int cap = o ? o->max_samples : 0;
    if (every > 0.0 && cap > samp_cap) {
      drop_graphs();
      samp_t.release(); samp_m.release();
      if (samp_t.alloc(cap) || samp_m.alloc((size_t)cap * 9)) {
        set_error("device allocation failed");
        return MMP_E_NOMEM;
      }
      samp_cap = cap;
    }
    Ctrl init{};
    init.fixed = 0;
    init.t_end = t_end;
    init.sample_every = every > 0.0 ? every : 0.0;
    init.t_next = every > 0.0 ? cur.t + every : t_end;
    if (init.t_next >= t_end - 1e-9 * (t_end - cur.t)) init.t_next = t_end;
    init.tol = p.tol > 0 ? p.tol : 1e-5;
    init.dt_min = p.dt_min > 0 ? p.dt_min : 1e-20;
    init.max_attempts = o ? o->max_steps : 0;
    if ((rc = begin_segment(init))) return rc;
    const bool sampling = every > 0.0;
    // enqueue attempts in chunks; the device ignores the ones after done
    const int chunk = N > 4096 ? 16 : 64;
    Ctrl c{};
    long long last = -1;
    while (true) {
      if ((rc = enqueue_attempts(false, sampling, chunk))) return rc;
      if ((rc = read_ctrl(&c))) return rc;
      if (c.done || c.status) break;
      const long long made = c.steps + c.rejects;
      if (made == last) {
        set_error("step controller made no progress");
        return MMP_E_STATE;
      }
      last = made;
    }
    if (info) {
      info->t = c.t; info->dt = c.dt; info->steps = c.steps; info->rejects = c.rejects;
      info->nsamples = c.nsamples; info->status = c.status;
    }
    if (sampling && o && c.nsamples > 0) {
      DeviceLock lk(device_mutex());
      const int ns = std::min(c.nsamples, samp_cap);
      std::vector<double> tt(ns), mm((size_t)ns * 9);
      MMP_HIP_TRY(hipMemcpy(tt.data(), samp_t.p, ns * sizeof(double), hipMemcpyDeviceToHost));
      MMP_HIP_TRY(hipMemcpy(mm.data(), samp_m.p, ns * 9 * sizeof(double), hipMemcpyDeviceToHost));
      for (int i = 0; i < ns; ++i) {
        if (o->sample_t) o->sample_t[i] = tt[i];
        if (o->sample_m)
          for (int q = 0; q < 3 * p.nsub; ++q) o->sample_m[i * 3 * p.nsub + q] = mm[i * 3 * p.nsub + q];
      }
    }
    if (c.status) {
      set_error(c.status == MMP_E_DT_UNDERFLOW ? "time step underflow" : "non-finite state");
      return c.status;
    }
    return 0;
  }

  int summary(double* m_avg, double* e) override {
    if (int rc = ensure_ready()) return rc;
    DeviceLock lk(device_mutex());
    if (!sctrl.p && (sctrl.alloc(1) || sres.alloc(10))) {
      set_error("device allocation failed");
      return MMP_E_NOMEM;
    }
    MMP_HIP_TRY(hipStreamSynchronize(stream));
    Ctrl c{};
    c.sample_pending = 1;
    MMP_HIP_TRY(hipMemcpy(sctrl.p, &c, sizeof(c), hipMemcpyHostToDevice));
    launch_sample<T>(sctrl.p, dtbl.p, p.nsub, N, spart.p, nsamp_blk, sres.p, sres.p + 1, 1,
                     stream, nullptr);
    MMP_HIP_TRY(hipGetLastError());
    if (int rc = eval(0, nullptr, e)) return rc;   // synchronises the stream
    MMP_HIP_TRY(hipMemcpy(m_avg, sres.p + 1, 3 * (size_t)p.nsub * sizeof(double),
                          hipMemcpyDeviceToHost));
    return 0;
  }

  int eval(uint32_t mask, double* b, double* e) override {
    int rc = ensure_ready();
    if (rc) return rc;
    const size_t nm = (size_t)p.nsub * 3 * N;
    Buf<T> bout;
    if (b && bout.alloc(nm)) { set_error("device allocation failed"); return MMP_E_NOMEM; }
    if (p.elastic) {
      ElasticArgs<T> ee = ea;
      ee.stage = 1;
      ee.ctrl = nullptr;
      launch_strain(ee, stream, &prof);
    }
    if (p.demag)
      demag_field<T>(plan, db, dtbl.p, 1, nullptr, (T)p.sub[0].Ms, ms_of(1), p.nsub, stream,
                     &prof, ms_of(2));
    FieldArgs<T> a = fa;
    a.ctrl = nullptr;
    a.stage = 1;
    a.mask = mask & MMP_T_ALL;
    a.add_zl = (mask & MMP_T_ZL) ? 1 : 0;
    a.out_torque = (mask & MMP_OUT_TORQUE) ? 1 : 0;
    a.bout = b ? bout.p : nullptr;
    a.epart = epart.p;
    launch_field<T>(a, true, stream, &prof);
    launch_energy_final(epart.p, nblk, eout.p, stream);
    double el = 0.0;
    if (p.elastic) {
      ElasticArgs<T> ee = ea;
      ee.stage = 1;
      ee.ctrl = nullptr;
      launch_elastic_stage<T>(ee, true, stream, &prof);
    }
    MMP_HIP_TRY(hipGetLastError());
    MMP_HIP_TRY(hipStreamSynchronize(stream));
    if (b) {
      std::vector<T> tmp(nm);
      MMP_HIP_TRY(hipMemcpy(tmp.data(), bout.p, nm * sizeof(T), hipMemcpyDeviceToHost));
      for (size_t i = 0; i < nm; ++i) b[i] = (double)tmp[i];
      bout.release();
    }
    if (e) {
      MMP_HIP_TRY(hipMemcpy(e, eout.p, kNE * sizeof(double), hipMemcpyDeviceToHost));
      if (p.elastic) {
        const size_t nb = (N + 255) / 256;
        std::vector<double> part(nb);
        MMP_HIP_TRY(hipMemcpy(part.data(), elpart.p, nb * sizeof(double), hipMemcpyDeviceToHost));
        for (double v : part) el += v;
      }
      e[kNE - 1] = el;
    }
    return 0;
  }

  // B of the selected terms (or the torque) in the grid's precision, widened
  // into the caller's FP64 device buffer; the grid keeps the precision-sized
  // output buffer from the first call on
  Buf<T> evalb;
  int eval_device(uint32_t mask, double* b) override {
    int rc = ensure_ready();
    if (rc) return rc;
    if ((rc = check_device_buffer(b, stream, "b"))) return rc;
    const size_t nm = (size_t)p.nsub * 3 * N;
    T* out = nullptr;
    if constexpr (sizeof(T) == sizeof(double)) {
      out = reinterpret_cast<T*>(b);
    } else {
      if (evalb.n < nm) {
        evalb.release();
        if (evalb.alloc(nm)) { set_error("device allocation failed"); return MMP_E_NOMEM; }
      }
      out = evalb.p;
    }
    if (p.elastic) {
      ElasticArgs<T> ee = ea;
      ee.stage = 1;
      ee.ctrl = nullptr;
      launch_strain(ee, stream, &prof);
    }
    if (p.demag)
      demag_field<T>(plan, db, dtbl.p, 1, nullptr, (T)p.sub[0].Ms, ms_of(1), p.nsub, stream,
                     &prof, ms_of(2));
    FieldArgs<T> a = fa;
    a.ctrl = nullptr;
    a.stage = 1;
    a.mask = mask & MMP_T_ALL;
    a.add_zl = (mask & MMP_T_ZL) ? 1 : 0;
    a.out_torque = (mask & MMP_OUT_TORQUE) ? 1 : 0;
    a.bout = out;
    a.epart = nullptr;
    launch_field<T>(a, true, stream, &prof);
    if constexpr (sizeof(T) != sizeof(double))
      hipLaunchKernelGGL(k_widen<T>, dim3(copy_blocks((long)nm)), dim3(256), 0, stream, out, b,
                         (long)nm);
    MMP_HIP_TRY(hipGetLastError());
    return 0;
  }

  // Chunks of the non-blocking run: each ends with an asynchronous copy of
  // the controller into a pinned slot of its own and an event, so two
  // chunks can be in flight while the host reads the older one.
  hipEvent_t chunk_ev[2] = {nullptr, nullptr};
  Ctrl* chunk_ctrl[2] = {nullptr, nullptr};
  int chunk_head = 0, chunk_count = 0;
  Ctrl chunk_last{};

  int run_begin(double t_end) override {
    int rc = ensure_ready();
    if (rc) return rc;
    Ctrl cur{};
    if ((rc = read_ctrl(&cur))) return rc;
    Ctrl init{};
    init.fixed = 0;
    init.t_end = t_end;
    init.t_next = t_end;
    init.tol = p.tol > 0 ? p.tol : 1e-5;
    init.dt_min = p.dt_min > 0 ? p.dt_min : 1e-20;
    if ((rc = begin_segment(init))) return rc;
    for (int i = 0; i < 2; ++i) {
      if (!chunk_ev[i]) MMP_HIP_TRY(hipEventCreateWithFlags(&chunk_ev[i], hipEventDisableTiming));
      if (!chunk_ctrl[i]) {
        DeviceLock lk(device_mutex());
        MMP_HIP_TRY(hipHostMalloc((void**)&chunk_ctrl[i], sizeof(Ctrl), 0));
      }
    }
    chunk_head = 0;
    chunk_count = 0;
    chunk_last = *hctrl;
    return 0;
  }

  int run_chunk(int attempts) override {
    if (chunk_count >= 2) { set_error("two chunks already in flight"); return MMP_E_STATE; }
    if (int rc = enqueue_attempts(false, false, attempts)) return rc;
    const int slot = (chunk_head + chunk_count) & 1;
    MMP_HIP_TRY(hipMemcpyAsync(chunk_ctrl[slot], dctrl.p, sizeof(Ctrl), hipMemcpyDeviceToHost,
                               stream));
    MMP_HIP_TRY(hipEventRecord(chunk_ev[slot], stream));
    ++chunk_count;
    return 0;
  }

  // state after the oldest chunk in flight (MMP_PENDING while it runs; the
  // last state read when none is in flight)
  int run_poll(bool* finished, int* status, long long* steps, long long* rejects) override {
    if (chunk_count > 0) {
      const hipError_t q = hipEventQuery(chunk_ev[chunk_head]);
      if (q == hipErrorNotReady) { *finished = false; return MMP_PENDING; }
      if (q != hipSuccess) { set_error(hipGetErrorString(q)); return MMP_E_HIP; }
      chunk_last = *chunk_ctrl[chunk_head];
      chunk_head ^= 1;
      --chunk_count;
    }
    const Ctrl& c = chunk_last;
    *finished = (c.done || c.status) != 0;
    *status = c.status;
    *steps = c.steps;
    *rejects = c.rejects;
    return 0;
  }

  int chunks_in_flight() const override { return chunk_count; }

  void set_chunk_state(const void* c) override {
    chunk_last = *static_cast<const Ctrl*>(c);
    chunk_count = 0;
  }

  int tensor(double* n6) override {
    double* d6 = nullptr;
    DeviceLock lk(device_mutex());
    MMP_HIP_TRY(hipMalloc(&d6, 6 * (size_t)N * sizeof(double)));
    const int rc = demag_tensor_only(nx, ny, nz, d[0], d[1], d[2], d6, stream);
    hipError_t e = hipStreamSynchronize(stream);
    if (rc == 0 && e == hipSuccess)
      e = hipMemcpy(n6, d6, 6 * (size_t)N * sizeof(double), hipMemcpyDeviceToHost);
    (void)hipFree(d6);
    if (rc || e != hipSuccess) { set_error("tensor build failed"); return MMP_E_HIP; }
    return 0;
  }
  // device address of the state slot of the pointer table
  const T* const* yn_slot() const {
    return reinterpret_cast<const T* const*>(reinterpret_cast<const char*>(dtbl.p) +
                                             offsetof(Table<T>, yn));
  }

  int stray_check(double height) {
    if (int rc = ensure_ready()) return rc;
    if (!(height >= 0.5 * d[2])) {
      set_error("stray field: height must be >= dz/2 (the layer clears the magnet)");
      return MMP_E_ARG;
    }
    return 0;
  }

  // tensor table into k6, then the field into dout, on the grid's stream
  hipError_t stray_launch(double height, double* k6, double* dout) {
    const double zt = (nz - 0.5) * d[2] + height;
    if (stray_kernel_build(nx, ny, nz, d[0], d[1], d[2], zt, k6, stream))
      return hipErrorLaunchFailure;
    launch_stray<T>(yn_slot(), p.nsub, p.sub[0].Ms, p.nsub >= 2 ? p.sub[1].Ms : 0.0,
                    p.nsub == 3 ? p.sub[2].Ms : 0.0, k6, nx, ny, nz, dout, stream);
    return hipGetLastError();
  }

  // stray field in the layer of cells centred `height` above the top
  // surface (synchronous; host output [3][ny][nx])
  int stray(double height, double* out) override {
    if (int rc = stray_check(height)) return rc;
    const size_t nk = (size_t)6 * nz * (2 * ny - 1) * (2 * nx - 1);
    const size_t no = (size_t)3 * nx * ny;
    double *k6 = nullptr, *dout = nullptr;
    DeviceLock lk(device_mutex());
    MMP_HIP_TRY(hipStreamSynchronize(stream));
    if (hipMalloc(&k6, nk * sizeof(double)) != hipSuccess) {
      set_error("stray field: device allocation failed");
      return MMP_E_NOMEM;
    }
    if (hipMalloc(&dout, no * sizeof(double)) != hipSuccess) {
      (void)hipFree(k6);
      set_error("stray field: device allocation failed");
      return MMP_E_NOMEM;
    }
    hipError_t e = stray_launch(height, k6, dout);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e == hipSuccess) e = hipMemcpy(out, dout, no * sizeof(double), hipMemcpyDeviceToHost);
    (void)hipFree(k6);
    (void)hipFree(dout);
    if (e != hipSuccess) {
      set_error(std::string("stray field: ") + hipGetErrorString(e));
      return MMP_E_HIP;
    }
    return 0;
  }

  // the same field into a caller-owned device buffer, the tensor table in
  // the library's fixed per-device table; enqueued on the grid's stream
  // with no allocation and no host synchronisation
  int stray_noalloc(double height, double* dout) override {
    if (int rc = stray_check(height)) return rc;
    const long nk = 6L * nz * (2L * ny - 1) * (2L * nx - 1);
    if (nk > kStrayScratchDoubles) {
      set_error("stray field (no allocation): the tensor table needs " + std::to_string(nk) +
                " doubles, above the fixed " + std::to_string(kStrayScratchDoubles) +
                " (6 nz (2nx-1)(2ny-1) must not exceed it)");
      return MMP_E_TOO_LARGE;
    }
    hipPointerAttribute_t at{};
    if (hipPointerGetAttributes(&at, dout) != hipSuccess || at.type != hipMemoryTypeDevice) {
      (void)hipGetLastError();
      set_error("stray field (no allocation): b_out_dev is not device memory");
      return MMP_E_ARG;
    }
    int dev = 0;
    MMP_HIP_TRY(hipStreamGetDevice(stream, &dev));
    if (at.device != dev) {
      set_error("stray field (no allocation): b_out_dev is on another device than the grid");
      return MMP_E_ARG;
    }
    double* k6 = nullptr;
    if (stray_scratch(dev, &k6)) {
      set_error("stray field (no allocation): hipGetSymbolAddress of the tensor table failed");
      return MMP_E_HIP;
    }
    MMP_HIP_TRY(stray_launch(height, k6, dout));
    return 0;
  }

};

GridBase* make_grid(int precision) {
  if (precision == MMP_FP64) return new Grid<double>();
  return new Grid<float>();
}

// gathers the members' controllers for one read-back
__global__ void k_gather_ctrl(Ctrl* const* __restrict__ src, Ctrl* __restrict__ dst, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = *src[i];
}

// Failure injection for host-side tests of the server's error handling:
// the next n batch rebuilds fail with MMP_E_NOMEM (no device work is done).
static std::atomic<int> g_batch_fail{0};
static bool batch_fail_injected() {
  int v = g_batch_fail.load();
  while (v > 0)
    if (g_batch_fail.compare_exchange_weak(v, v - 1)) return true;
  return false;
}

template <typename T>
struct Batch final : BatchBase {
  int nsub;
  std::vector<Grid<T>*> mem;
  hipStream_t st = nullptr;
  // device tables (rebuilt when membership changes)
  Buf<FieldArgs<T>> d_args;
  Buf<int2> d_work;
  DemagMulti<T> dm;  // demag passes of the members with demag
  Buf<StepWork<T>> d_step;
  Buf<Ctrl*> d_cptr;
  Buf<Ctrl> d_cgather;
  int nwork = 0;
  long max_cells = 0;
  bool dirty = true;
  hipGraphExec_t gexec = nullptr;
  static constexpr int kGA = 8;
  // two read-back slots
  Ctrl* h_c[2] = {nullptr, nullptr};
  int h_cap = 0;
  hipEvent_t ev[2] = {nullptr, nullptr};
  int head = 0, count = 0;
  std::vector<Grid<T>*> slot_mem[2];

  explicit Batch(int ns) : nsub(ns) {}
  ~Batch() override {
    if (st) (void)hipStreamSynchronize(st);
    DeviceLock lk(device_mutex());
    if (gexec) (void)hipGraphExecDestroy(gexec);
    for (int i = 0; i < 2; ++i) {
      if (h_c[i]) (void)hipHostFree(h_c[i]);
      if (ev[i]) (void)hipEventDestroy(ev[i]);
    }
    if (st) (void)hipStreamDestroy(st);
  }

  bool accepts(const GridBase* g) const override {
    const auto* t = dynamic_cast<const Grid<T>*>(g);
    // one stage sequence serves every member: the Dormand-Prince pair; a
    // member with demag joins the batched demag passes (open boundaries,
    // lines that fit one block of the LDS kernels)
    if (!t || !t->params_set || t->p.elastic || t->p.nsub != nsub || t->p.solver != RK_DP45 ||
        t->p.bc_eq6 || (t->p.ngrains > 0 && t->p.grain_exch_reduction != 0.0))
      return false;
    if (t->p.demag)
      return t->demag_built && t->p.pbc[0] == 0 && t->p.pbc[1] == 0 && demag_multi_fits(t->plan);
    return true;
  }
  int size() const override { return (int)mem.size(); }
  int in_flight() const override { return count; }
  long long cells() const override {
    long long c = 0;
    for (auto* g : mem) c += g->N * g->p.nsub;
    return c;
  }

  int ensure_stream() {
    if (!st) {
      DeviceLock lk(device_mutex());
      MMP_HIP_TRY(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    }
    for (int i = 0; i < 2; ++i)
      if (!ev[i]) MMP_HIP_TRY(hipEventCreateWithFlags(&ev[i], hipEventDisableTiming));
    return 0;
  }

  int add(GridBase* gb) override {
    if (count) { set_error("batch membership changes need an idle batch"); return MMP_E_STATE; }
    auto* g = dynamic_cast<Grid<T>*>(gb);
    if (!g || !accepts(g)) { set_error("grid cannot join this batch"); return MMP_E_ARG; }
    if (int rc = ensure_stream()) return rc;
    // the batch stream waits for the member's set-up (run_begin)
    hipEvent_t e;
    MMP_HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    MMP_HIP_TRY(hipEventRecord(e, g->stream));
    MMP_HIP_TRY(hipStreamWaitEvent(st, e, 0));
    (void)hipEventDestroy(e);
    mem.push_back(g);
    dirty = true;
    return 0;
  }

  int remove(GridBase* gb) override {
    if (count) { set_error("batch membership changes need an idle batch"); return MMP_E_STATE; }
    for (size_t i = 0; i < mem.size(); ++i)
      if (mem[i] == gb) {
        mem.erase(mem.begin() + i);
        dirty = true;
        return 0;
      }
    return MMP_E_ARG;
  }

  int rebuild() {
    if (batch_fail_injected()) {
      set_error("batch rebuild failed (injected)");
      return MMP_E_NOMEM;
    }
    if (gexec) {
      (void)hipGraphExecDestroy(gexec);
      gexec = nullptr;
    }
    const int n = (int)mem.size();
    std::vector<FieldArgs<T>> args(n);
    std::vector<int2> work;
    std::vector<StepWork<T>> step(n);
    std::vector<Ctrl*> cptr(n);
    max_cells = 0;
    for (int i = 0; i < n; ++i) {
      Grid<T>* g = mem[i];
      args[i] = g->fa;
      for (int b = 0; b < g->nblk; ++b) work.push_back(make_int2(i, b));
      step[i].ctrl = g->dctrl.p;
      step[i].tbl = g->dtbl.p;
      step[i].errpart = g->errpart.p;
      step[i].nerr = g->nblk;
      step[i].nsub = g->p.nsub;
      step[i].N = g->N;
      cptr[i] = g->dctrl.p;
      max_cells = std::max(max_cells, (long)g->N * g->p.nsub);
    }
    nwork = (int)work.size();
    {
      std::vector<DemagMember<T>> dms;
      for (Grid<T>* g : mem)
        if (g->p.demag)
          dms.push_back({&g->plan, g->db, g->dtbl.p, g->dctrl.p, (T)g->p.sub[0].Ms, g->ms_of(1),
                         g->ms_of(2), g->p.nsub});
      if (int rc = dm.build(dms, st)) return rc;
    }
    d_args.release(); d_work.release(); d_step.release(); d_cptr.release(); d_cgather.release();
    if (d_args.alloc(n) || d_work.alloc(work.size()) || d_step.alloc(n) || d_cptr.alloc(n) ||
        d_cgather.alloc(n)) {
      set_error("device allocation failed");
      return MMP_E_NOMEM;
    }
    MMP_HIP_TRY(hipMemcpyAsync(d_args.p, args.data(), n * sizeof(FieldArgs<T>),
                               hipMemcpyHostToDevice, st));
    MMP_HIP_TRY(hipMemcpyAsync(d_work.p, work.data(), work.size() * sizeof(int2),
                               hipMemcpyHostToDevice, st));
    MMP_HIP_TRY(hipMemcpyAsync(d_step.p, step.data(), n * sizeof(StepWork<T>),
                               hipMemcpyHostToDevice, st));
    MMP_HIP_TRY(hipMemcpyAsync(d_cptr.p, cptr.data(), n * sizeof(Ctrl*), hipMemcpyHostToDevice,
                               st));
    MMP_HIP_TRY(hipStreamSynchronize(st));  // host vectors go out of scope
    if (n > h_cap) {
      DeviceLock lk(device_mutex());
      for (int i = 0; i < 2; ++i) {
        if (h_c[i]) (void)hipHostFree(h_c[i]);
        h_c[i] = nullptr;
        MMP_HIP_TRY(hipHostMalloc((void**)&h_c[i], n * sizeof(Ctrl), 0));
      }
      h_cap = n;
    }
    dirty = false;
    return 0;
  }

  void attempt() {
    constexpr int ns = RK::t[RK_DP45].ns;
    for (int s = 2; s <= ns; ++s) {
      dm.launch(s, st);
      launch_field_multi<T>(d_args.p, d_work.p, nwork, nsub, s, 0, st);
    }
    launch_step_multi<T>(d_step.p, (int)mem.size(), max_cells, st);
  }

  int run_chunk(int attempts) override {
    if (mem.empty()) return 0;
    if (count >= 2) { set_error("two chunks already in flight"); return MMP_E_STATE; }
    if (dirty) {
      if (int rc = rebuild()) return rc;
    }
    int left = attempts;
    if (left >= kGA) {
      if (!gexec) {
        DeviceLock lk(device_mutex());
        hipGraph_t g = nullptr;
        MMP_HIP_TRY(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
        for (int i = 0; i < kGA; ++i) attempt();
        const hipError_t e = hipStreamEndCapture(st, &g);
        if (e != hipSuccess) {
          if (g) (void)hipGraphDestroy(g);
          set_error(std::string("batch graph capture: ") + hipGetErrorString(e));
          return MMP_E_HIP;
        }
        const hipError_t e2 = hipGraphInstantiate(&gexec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e2 != hipSuccess) {
          gexec = nullptr;
          set_error(std::string("batch graph instantiate: ") + hipGetErrorString(e2));
          return MMP_E_HIP;
        }
      }
      for (; left >= kGA; left -= kGA) MMP_HIP_TRY(hipGraphLaunch(gexec, st));
    }
    for (; left > 0; --left) attempt();
    const int n = (int)mem.size();
    const int slot = (head + count) & 1;
    hipLaunchKernelGGL(k_gather_ctrl, dim3((n + 63) / 64), dim3(64), 0, st, d_cptr.p, d_cgather.p,
                       n);
    MMP_HIP_TRY(hipGetLastError());
    MMP_HIP_TRY(hipMemcpyAsync(h_c[slot], d_cgather.p, n * sizeof(Ctrl), hipMemcpyDeviceToHost, st));
    MMP_HIP_TRY(hipEventRecord(ev[slot], st));
    slot_mem[slot] = mem;
    ++count;
    return 0;
  }

  void abandon() override {
    if (st) (void)hipStreamSynchronize(st);
    (void)hipGetLastError();
    count = 0;
    head = 0;
    for (auto& v : slot_mem) v.clear();
    mem.clear();
    dirty = true;
    if (gexec) {
      (void)hipGraphExecDestroy(gexec);
      gexec = nullptr;
    }
  }

  int poll() override {
    if (count == 0) return 0;
    const hipError_t q = hipEventQuery(ev[head]);
    if (q == hipErrorNotReady) return MMP_PENDING;
    if (q != hipSuccess) { set_error(hipGetErrorString(q)); return MMP_E_HIP; }
    const std::vector<Grid<T>*>& m = slot_mem[head];
    for (size_t i = 0; i < m.size(); ++i) m[i]->set_chunk_state(&h_c[head][i]);
    head ^= 1;
    --count;
    return 0;
  }
};

extern "C" void mmp_test_fail_batch_rebuilds(int n) { g_batch_fail.store(n < 0 ? 0 : n); }

BatchBase* make_batch(int precision, int nsub) {
  if (precision == MMP_FP64) return new Batch<double>(nsub);
  return new Batch<float>(nsub);
}

}  // namespace mmp
