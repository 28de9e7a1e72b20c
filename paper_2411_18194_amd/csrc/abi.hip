// extern "C" surface of libmmp (declared in include/mmp.h).
#include <cstring>
#include <exception>
#include <new>
#include <string>

#include "grid.h"

namespace mmp {

static thread_local std::string g_last_error;
std::recursive_mutex& device_mutex() {
  static std::recursive_mutex mu;
  return mu;
}
void set_error(const std::string& msg) { g_last_error = msg; }
const char* get_error() { return g_last_error.c_str(); }

const char* const kProfNames[P_COUNT] = {
    "fftx_fwd", "ffty_fwd", "fftz_mul", "ffty_inv", "fftx_inv", "ffty_mul2d",
    "field",    "combine",  "control",  "elastic",  "reduce"};

hipEvent_t Prof::get() {
  if (!pool.empty()) {
    hipEvent_t e = pool.back();
    pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  (void)hipEventCreate(&e);
  return e;
}
void Prof::begin(int, hipStream_t s, hipEvent_t* a) {
  *a = get();
  (void)hipEventRecord(*a, s);
}
void Prof::end(int id, hipStream_t s, hipEvent_t a) {
  hipEvent_t b = get();
  (void)hipEventRecord(b, s);
  pending.push_back({id, a, b});
  if (pending.size() > 4096) resolve();
}
void Prof::resolve() {
  for (auto& q : pending) {
    (void)hipEventSynchronize(q.b);
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, q.a, q.b) == hipSuccess) {
      total_ms[q.id] += ms;
      count[q.id] += 1;
    }
    pool.push_back(q.a);
    pool.push_back(q.b);
  }
  pending.clear();
}
void Prof::reset() {
  resolve();
  for (int i = 0; i < P_COUNT; ++i) { total_ms[i] = 0; count[i] = 0; }
}
Prof::~Prof() {
  for (auto& q : pending) {
    (void)hipEventDestroy(q.a);
    (void)hipEventDestroy(q.b);
  }
  for (auto e : pool) (void)hipEventDestroy(e);
}

}  // namespace mmp

using namespace mmp;

#define MMP_GUARD_BEGIN try {
#define MMP_GUARD_END                                    \
  }                                                      \
  catch (const std::bad_alloc&) {                        \
    set_error("host allocation failed");                 \
    return MMP_E_NOMEM;                                  \
  }                                                      \
  catch (const std::exception& ex) {                     \
    set_error(ex.what());                                \
    return MMP_E_ARG;                                    \
  }                                                      \
  catch (...) {                                          \
    set_error("unknown error");                          \
    return MMP_E_ARG;                                    \
  }

static int check_grid(mmp_grid g) {
  if (!g) { set_error("null grid"); return MMP_E_ARG; }
  if (!g->impl) { set_error("mmp_set_params has not been called"); return MMP_E_STATE; }
  return 0;
}

extern "C" {

const char* mmp_last_error(void) { return get_error(); }

mmp_status mmp_grid_create(int32_t nx, int32_t ny, int32_t nz, const double cellsize[3],
                           mmp_grid* out) {
  MMP_GUARD_BEGIN
  if (!out) { set_error("null output handle"); return MMP_E_ARG; }
  *out = nullptr;
  if (nx < 1 || ny < 1 || nz < 1) { set_error("grid sizes must be >= 1"); return MMP_E_ARG; }
  if ((long long)nx * ny * nz > (1LL << 31) / 8) { set_error("grid too large"); return MMP_E_ARG; }
  if (!cellsize || !(cellsize[0] > 0) || !(cellsize[1] > 0) || !(cellsize[2] > 0)) {
    set_error("cell sizes must be > 0");
    return MMP_E_ARG;
  }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
    set_error("no HIP device available");
    return MMP_E_HIP;
  }
  mmp_grid g = new mmp_grid_s();
  g->nx = nx; g->ny = ny; g->nz = nz;
  for (int i = 0; i < 3; ++i) g->d[i] = cellsize[i];
  *out = g;
  return MMP_OK;
  MMP_GUARD_END
}

mmp_status mmp_grid_destroy(mmp_grid g) {
  MMP_GUARD_BEGIN
  if (!g) return MMP_OK;
  if (g->impl) {
    (void)hipStreamSynchronize(g->impl->stream);
    hipStream_t own = g->impl->own_stream;
    g->impl.reset();
    if (own) {
      DeviceLock lk(device_mutex());
      (void)hipStreamDestroy(own);
    }
  }
  delete g;
  return MMP_OK;
  MMP_GUARD_END
}

mmp_status mmp_set_params(mmp_grid g, const mmp_params* p) {
  MMP_GUARD_BEGIN
  DeviceLock lk(device_mutex());  // synchronous copies: not during a capture
  if (!g || !p) { set_error("null argument"); return MMP_E_ARG; }
  if (p->struct_size != sizeof(mmp_params)) { set_error("mmp_params struct_size mismatch"); return MMP_E_ARG; }
  if (p->precision != MMP_FP32 && p->precision != MMP_FP64) { set_error("bad precision"); return MMP_E_ARG; }
  if (p->nsub < 1 || p->nsub > 3) { set_error("nsub must be 1, 2 or 3"); return MMP_E_ARG; }
  if (p->nsub == 3 && (p->elastic || p->bc_eq6 || p->dmi_homo[0] != 0.0 ||
                       p->dmi_homo[1] != 0.0 || p->dmi_homo[2] != 0.0)) {
    set_error("three sublattices: open boundaries, no elasticity, no homogeneous DMI");
    return MMP_E_ARG;
  }
  if (p->solver < 0 || p->solver >= RK_COUNT) { set_error("unknown solver"); return MMP_E_ARG; }
  if (p->pbc[0] < 0 || p->pbc[1] < 0 || p->pbc[0] > 1024 || p->pbc[1] > 1024 || p->pbc[2] != 0) {
    set_error("pbc: repetitions 0..1024 along x and y, 0 along z");
    return MMP_E_ARG;
  }
  if ((p->pbc[0] || p->pbc[1]) && p->elastic) {
    set_error("periodic boundaries are not combined with elasticity");
    return MMP_E_ARG;
  }
  if (p->ngrains < 0 || p->ngrains > 65536 || (p->ngrains > 0 && (!p->grain || !p->grain_axes))) {
    set_error("bad grain description");
    return MMP_E_ARG;
  }
  {
    const double fmn = p->fac_min > 0 ? p->fac_min : 0.1, fmx = p->fac_max > 0 ? p->fac_max : 2.0;
    // fac_min < 1: a rejected attempt must shrink the step, or an adaptive
    // run retries the same step forever
    if (!(p->dt_max >= 0.0) || !(p->safety >= 0.0 && p->safety <= 1.0) ||
        !(p->fac_min >= 0.0 && p->fac_min < 1.0) || !(p->fac_max == 0.0 || p->fac_max >= 1.0) ||
        !(fmn <= fmx)) {
      set_error("step control: dt_max >= 0, safety in (0, 1], fac_min in (0, 1), fac_max >= 1");
      return MMP_E_ARG;
    }
  }
  if (!(p->grain_exch_reduction >= 0.0 && p->grain_exch_reduction <= 1.0)) {
    set_error("grain_exch_reduction must be in [0, 1]");
    return MMP_E_ARG;
  }
  if (p->nsub == 2 && p->A0 != 0.0 && !(p->latcon > 0)) { set_error("latcon must be > 0"); return MMP_E_ARG; }
  if (p->elastic && !(p->rho > 0)) { set_error("rho must be > 0"); return MMP_E_ARG; }
  if (!(p->rayleigh >= 0.0)) { set_error("rayleigh must be >= 0"); return MMP_E_ARG; }
  {
    bool tens = false;
    for (int s = 0; s < 2; ++s)
      for (int i = 0; i < 3; ++i)
        for (int c = 0; c < 3; ++c)
          tens = tens || p->dmi_W[s][i][c] != 0.0 || (s == 0 && p->dmi_W12[i][c] != 0.0);
    if (tens && !p->bc_eq6) {
      set_error("DMI tensors need the Eq. 6 boundary condition (bc_eq6 = 1)");
      return MMP_E_ARG;
    }
    if (p->bc_eq6 && (p->sub[0].Dint != 0.0 || (p->nsub >= 2 && p->sub[1].Dint != 0.0))) {
      set_error("with bc_eq6 give the interfacial DMI as a tensor");
      return MMP_E_ARG;
    }
  }
  if (p->dmi_layer < -1 || p->dmi_layer >= g->nz) { set_error("bad dmi_layer"); return MMP_E_ARG; }
  const long N = (long)g->nx * g->ny * g->nz;
  if (p->ngrains > 0)
    for (long i = 0; i < N; ++i)
      if (p->grain[i] >= p->ngrains) { set_error("grain id out of range"); return MMP_E_ARG; }
  if (!g->impl || g->impl->precision != p->precision) {
    hipStream_t keep = g->user_stream;
    if (g->impl) {
      (void)hipStreamSynchronize(g->impl->stream);
      hipStream_t own = g->impl->own_stream;
      g->impl.reset();
      if (own) {
        DeviceLock lk(device_mutex());
        (void)hipStreamDestroy(own);
      }
    }
    GridBase* b = make_grid(p->precision);
    b->nx = g->nx; b->ny = g->ny; b->nz = g->nz;
    for (int i = 0; i < 3; ++i) b->d[i] = g->d[i];
    b->N = N;
    b->precision = p->precision;
    hipError_t se;
    {
      DeviceLock lk(device_mutex());
      se = hipStreamCreateWithFlags(&b->own_stream, hipStreamNonBlocking);
    }
    if (se != hipSuccess) {
      delete b;
      set_error("stream creation failed");
      return MMP_E_HIP;
    }
    b->stream = keep ? keep : b->own_stream;
    g->impl.reset(b);
  }
  GridBase* b = g->impl.get();
  (void)hipStreamSynchronize(b->stream);
  const int old_nsub = b->params_set ? b->p.nsub : -1;
  b->p = *p;
  b->nsub = p->nsub;
  if (p->ngrains > 0) {
    b->grain.assign(p->grain, p->grain + N);
    b->grain_axes.assign(p->grain_axes, p->grain_axes + 3 * (size_t)p->ngrains);
  } else {
    b->grain.clear();
    b->grain_axes.clear();
  }
  b->p.grain = nullptr;
  b->p.grain_axes = nullptr;
  (void)old_nsub;
  return b->apply_params();
  MMP_GUARD_END
}

mmp_status mmp_set_state(mmp_grid g, const double* m, const double* u, const double* v, double t) {
  MMP_GUARD_BEGIN
  DeviceLock lk(device_mutex());  // synchronous copies: not during a capture
  int rc = check_grid(g);
  if (rc) return rc;
  if (!m) { set_error("null magnetisation"); return MMP_E_ARG; }
  return g->impl->set_state(m, u, v, t);
  MMP_GUARD_END
}

mmp_status mmp_get_state(mmp_grid g, double* m, double* u, double* v, double* t, double* dt) {
  MMP_GUARD_BEGIN
  DeviceLock lk(device_mutex());  // synchronous copies: not during a capture
  int rc = check_grid(g);
  if (rc) return rc;
  if (!g->impl->state_set) { set_error("mmp_set_state has not been called"); return MMP_E_STATE; }
  return g->impl->get_state(m, u, v, t, dt);
  MMP_GUARD_END
}

mmp_status mmp_eval_heff(mmp_grid g, uint32_t mask, double* b, double* e) {
  MMP_GUARD_BEGIN
  DeviceLock lk(device_mutex());  // synchronous copies: not during a capture
  int rc = check_grid(g);
  if (rc) return rc;
  return g->impl->eval(mask, b, e);
  MMP_GUARD_END
}

mmp_status mmp_set_state_device(mmp_grid g, const double* m_dev, const double* u_dev,
                                const double* v_dev, double t) {
  MMP_GUARD_BEGIN
  int rc = check_grid(g);
  if (rc) return rc;
  if (!m_dev) { set_error("null magnetisation"); return MMP_E_ARG; }
  return g->impl->set_state_device(m_dev, u_dev, v_dev, t);
  MMP_GUARD_END
}

mmp_status mmp_get_state_device(mmp_grid g, double* m_dev, double* u_dev, double* v_dev,
                                double* t_dt_dev) {
  MMP_GUARD_BEGIN
  int rc = check_grid(g);
  if (rc) return rc;
  if (!g->impl->state_set) { set_error("mmp_set_state has not been called"); return MMP_E_STATE; }
  return g->impl->get_state_device(m_dev, u_dev, v_dev, t_dt_dev);
  MMP_GUARD_END
}

mmp_status mmp_eval_heff_device(mmp_grid g, uint32_t mask, double* b_dev) {
  MMP_GUARD_BEGIN
  int rc = check_grid(g);
  if (rc) return rc;
  if (!b_dev) { set_error("null output"); return MMP_E_ARG; }
  return g->impl->eval_device(mask, b_dev);
  MMP_GUARD_END
}

mmp_status mmp_step(mmp_grid g, double dt_fixed, mmp_step_info* info) {
  MMP_GUARD_BEGIN
  int rc = check_grid(g);
  if (rc) return rc;
  if (dt_fixed < 0) { set_error("dt_fixed must be >= 0"); return MMP_E_ARG; }
  return g->impl->step(dt_fixed, info);
  MMP_GUARD_END
}

mmp_status mmp_run_fixed(mmp_grid g, double dt, int64_t nsteps, mmp_step_info* info) {
  MMP_GUARD_BEGIN
  int rc = check_grid(g);
  if (rc) return rc;
  return g->impl->run_fixed(dt, nsteps, info);
  MMP_GUARD_END
}

mmp_status mmp_run(mmp_grid g, double t_end, const mmp_run_opts* o, mmp_run_info* info) {
  MMP_GUARD_BEGIN
  int rc = check_grid(g);
  if (rc) return rc;
  if (o && o->struct_size != sizeof(mmp_run_opts)) { set_error("mmp_run_opts struct_size mismatch"); return MMP_E_ARG; }
  if (o && (o->sample_every < 0 || o->max_samples < 0)) { set_error("bad sampling options"); return MMP_E_ARG; }
  if (o && o->sample_every > 0 && (!o->sample_t && !o->sample_m)) { set_error("sampling needs output buffers"); return MMP_E_ARG; }
  return g->impl->run(t_end, o, info);
  MMP_GUARD_END
}

mmp_status mmp_set_stream(mmp_grid g, void* s) {
  MMP_GUARD_BEGIN
  if (!g) { set_error("null grid"); return MMP_E_ARG; }
  g->user_stream = (hipStream_t)s;
  if (g->impl) {
    (void)hipStreamSynchronize(g->impl->stream);
    g->impl->stream = s ? (hipStream_t)s : g->impl->own_stream;
  }
  return MMP_OK;
  MMP_GUARD_END
}

mmp_status mmp_set_graphs(mmp_grid g, int32_t on) {
  MMP_GUARD_BEGIN
  if (int rc = check_grid(g)) return rc;
  (void)hipStreamSynchronize(g->impl->stream);
  return g->impl->set_graphs(on != 0);
  MMP_GUARD_END
}

mmp_status mmp_synchronize(mmp_grid g) {
  MMP_GUARD_BEGIN
  int rc = check_grid(g);
  if (rc) return rc;
  MMP_HIP_TRY(hipStreamSynchronize(g->impl->stream));
  return MMP_OK;
  MMP_GUARD_END
}

mmp_status mmp_grid_bytes(mmp_grid g, int64_t* bytes) {
  MMP_GUARD_BEGIN
  int rc = check_grid(g);
  if (rc) return rc;
  if (!bytes) { set_error("null output"); return MMP_E_ARG; }
  *bytes = g->impl->bytes();
  return MMP_OK;
  MMP_GUARD_END
}

mmp_status mmp_get_demag_tensor(mmp_grid g, double* n6) {
  MMP_GUARD_BEGIN
  DeviceLock lk(device_mutex());  // synchronous copies: not during a capture
  int rc = check_grid(g);
  if (rc) return rc;
  if (!n6) { set_error("null output"); return MMP_E_ARG; }
  return g->impl->tensor(n6);
  MMP_GUARD_END
}

mmp_status mmp_stray_field(mmp_grid g, double height, double* b_out) {
  MMP_GUARD_BEGIN
  DeviceLock lk(device_mutex());  // synchronous copies: not during a capture
  int rc = check_grid(g);
  if (rc) return rc;
  if (!b_out) { set_error("null output"); return MMP_E_ARG; }
  return g->impl->stray(height, b_out);
  MMP_GUARD_END
}

mmp_status mmp_stray_field_noalloc(mmp_grid g, double height, double* b_out_dev) {
  MMP_GUARD_BEGIN
  int rc = check_grid(g);
  if (rc) return rc;
  if (!b_out_dev) { set_error("null output"); return MMP_E_ARG; }
  return g->impl->stray_noalloc(height, b_out_dev);
  MMP_GUARD_END
}

mmp_status mmp_get_plan(mmp_grid g, mmp_plan* out) {
  MMP_GUARD_BEGIN
  if (int rc = check_grid(g)) return rc;
  if (!out || out->struct_size != sizeof(mmp_plan)) {
    set_error("mmp_plan: null or struct_size mismatch");
    return MMP_E_ARG;
  }
  return g->impl->get_plan(out);
  MMP_GUARD_END
}

mmp_status mmp_set_plan(mmp_grid g, const mmp_plan* p) {
  MMP_GUARD_BEGIN
  DeviceLock lk(device_mutex());  // synchronous copies: not during a capture
  if (int rc = check_grid(g)) return rc;
  if (!p || p->struct_size != sizeof(mmp_plan)) {
    set_error("mmp_plan: null or struct_size mismatch");
    return MMP_E_ARG;
  }
  return g->impl->set_plan(p);
  MMP_GUARD_END
}

mmp_status mmp_autotune(mmp_grid g, mmp_plan* out) {
  MMP_GUARD_BEGIN
  DeviceLock lk(device_mutex());  // synchronous copies: not during a capture
  if (int rc = check_grid(g)) return rc;
  if (out && out->struct_size != sizeof(mmp_plan)) {
    set_error("mmp_plan: struct_size mismatch");
    return MMP_E_ARG;
  }
  return g->impl->autotune(out);
  MMP_GUARD_END
}

mmp_status mmp_prof_enable(mmp_grid g, int32_t on) {
  MMP_GUARD_BEGIN
  int rc = check_grid(g);
  if (rc) return rc;
  g->impl->prof.on = on != 0;
  return MMP_OK;
  MMP_GUARD_END
}

int32_t mmp_prof_count(void) { return P_COUNT; }

mmp_status mmp_prof_read(mmp_grid g, int32_t idx, const char** name, double* total_ms,
                         int64_t* launches) {
  MMP_GUARD_BEGIN
  int rc = check_grid(g);
  if (rc) return rc;
  if (idx < 0 || idx >= P_COUNT) { set_error("bad kernel class index"); return MMP_E_ARG; }
  g->impl->prof.resolve();
  if (name) *name = kProfNames[idx];
  if (total_ms) *total_ms = g->impl->prof.total_ms[idx];
  if (launches) *launches = g->impl->prof.count[idx];
  return MMP_OK;
  MMP_GUARD_END
}

mmp_status mmp_prof_reset(mmp_grid g) {
  MMP_GUARD_BEGIN
  int rc = check_grid(g);
  if (rc) return rc;
  g->impl->prof.reset();
  return MMP_OK;
  MMP_GUARD_END
}

}  // extern "C"
