// Host-side exercise of libmmp's C ABI under AddressSanitizer and
// UndefinedBehaviorSanitizer, with no GPU present: argument validation of
// every entry point, and a server's full life (worker and builder threads,
// admission, set-up failure of every request for want of a device, results
// handed out once, shutdown with requests still queued).  Built from the
// library's sources with the host code instrumented; exits non-zero on the
// first unexpected status (the sanitizers abort on their own findings).
#include <cstdio>
#include <cstring>
#include <vector>

#include "mmp.h"

static int fails = 0;
#define EXPECT(cond)                                              \
  do {                                                            \
    if (!(cond)) {                                                \
      std::fprintf(stderr, "%s:%d: %s\n", __FILE__, __LINE__, #cond); \
      ++fails;                                                    \
    }                                                             \
  } while (0)

int main() {
  // grids: bad sizes, bad cells, null handles
  mmp_grid g = nullptr;
  const double cs[3] = {1e-9, 1e-9, 1e-9}, bad[3] = {1e-9, -1.0, 1e-9};
  EXPECT(mmp_grid_create(0, 4, 4, cs, &g) == MMP_E_ARG);
  EXPECT(mmp_grid_create(4, 4, 4, bad, &g) == MMP_E_ARG);
  EXPECT(mmp_grid_create(4, 4, 4, cs, nullptr) == MMP_E_ARG);
  EXPECT(mmp_grid_create(1 << 12, 1 << 12, 1 << 12, cs, &g) == MMP_E_ARG);
  EXPECT(std::strlen(mmp_last_error()) > 0);
  const int rc = mmp_grid_create(4, 4, 4, cs, &g);
  EXPECT(rc == MMP_OK || rc == MMP_E_HIP);   // MMP_E_HIP: no device here
  EXPECT(mmp_set_params(nullptr, nullptr) == MMP_E_ARG);
  EXPECT(mmp_set_state(nullptr, nullptr, nullptr, nullptr, 0.0) == MMP_E_ARG);
  EXPECT(mmp_eval_heff(nullptr, 0, nullptr, nullptr) == MMP_E_ARG);
  EXPECT(mmp_step(nullptr, 0.0, nullptr) == MMP_E_ARG);
  EXPECT(mmp_run(nullptr, 1e-9, nullptr, nullptr) == MMP_E_ARG);
  EXPECT(mmp_stray_field(nullptr, 1e-9, nullptr) == MMP_E_ARG);
  EXPECT(mmp_stray_field_noalloc(nullptr, 1e-9, nullptr) == MMP_E_ARG);
  mmp_plan pl{};
  pl.struct_size = sizeof(pl);
  EXPECT(mmp_get_plan(nullptr, &pl) == MMP_E_ARG);
  EXPECT(mmp_autotune(nullptr, nullptr) == MMP_E_ARG);
  EXPECT(mmp_grid_destroy(nullptr) == MMP_OK);
  if (rc == MMP_OK) EXPECT(mmp_grid_destroy(g) == MMP_OK);

  // server: bad options, then a full life without a device
  mmp_server s = nullptr;
  mmp_server_opts o{};
  o.struct_size = sizeof(o);
  EXPECT(mmp_server_create(&o, &s) == MMP_E_ARG);    // no budget
  o.hbm_budget = 1 << 30;
  o.max_active = 2;
  o.precision = MMP_FP32;
  o.batch = 1;
  EXPECT(mmp_server_create(&o, &s) == MMP_OK);
  const int nx = 8, ny = 6, nz = 1;
  std::vector<double> m0(2 * 3 * nx * ny * nz, 0.0);
  for (int i = 0; i < nx * ny * nz; ++i) {
    m0[2 * nx * ny * nz + i] = 1.0;             // sublattice 1 along z
    m0[3 * nx * ny * nz + 2 * nx * ny * nz + i] = -1.0;
  }
  mmp_request r{};
  r.struct_size = sizeof(r);
  r.nx = nx; r.ny = ny; r.nz = nz;
  r.cellsize[0] = r.cellsize[1] = r.cellsize[2] = 1e-9;
  r.params.struct_size = sizeof(mmp_params);
  r.params.nsub = 2;
  r.params.gamma = 1.7595e11;
  r.params.sub[0].Ms = r.params.sub[1].Ms = 4e5;
  r.params.sub[0].A11 = r.params.sub[1].A11 = 1e-11;
  r.params.sub[0].alpha = r.params.sub[1].alpha = 0.05;
  r.params.A0 = -2.5e-11;
  r.params.latcon = 0.35e-9;
  r.params.dmi_layer = -1;
  r.params.tol = 1e-5;
  r.m0 = m0.data();
  r.t_relax = 1e-12;
  uint64_t t = 0;
  mmp_request badr = r;
  badr.nx = 0;
  EXPECT(mmp_submit(s, &badr, &t) == MMP_E_ARG);
  badr = r;
  badr.m0 = nullptr;
  EXPECT(mmp_submit(s, &badr, &t) == MMP_E_ARG);
  mmp_request huge = r;
  huge.nx = 4096; huge.ny = 4096;
  std::vector<double> mh((size_t)2 * 3 * 4096 * 4096, 0.0);
  huge.m0 = mh.data();
  EXPECT(mmp_submit(s, &huge, &t) == MMP_E_TOO_LARGE);
  std::vector<uint64_t> tickets;
  for (int k = 0; k < 6; ++k) {
    EXPECT(mmp_submit(s, &r, &t) == MMP_OK);
    tickets.push_back(t);
  }
  mmp_result res{};
  EXPECT(mmp_poll(s, 987654321, &res) == MMP_E_TICKET);
  // every request fails its set-up without a device; each result is handed
  // out exactly once
  int got = 0;
  for (int spin = 0; spin < 200000 && got < (int)tickets.size(); ++spin)
    for (uint64_t& tk : tickets) {
      if (!tk) continue;
      const int pr = mmp_poll(s, tk, &res);
      if (pr == MMP_OK) {
        EXPECT(res.status < 0);
        EXPECT(res.t_done >= res.t_admit && res.t_admit >= res.t_submit);
        EXPECT(mmp_poll(s, tk, &res) == MMP_E_TICKET);
        tk = 0;
        ++got;
      } else {
        EXPECT(pr == MMP_PENDING);
      }
    }
  EXPECT(got == (int)tickets.size());
  // shutdown with requests still queued
  for (int k = 0; k < 4; ++k) EXPECT(mmp_submit(s, &r, &t) == MMP_OK);
  EXPECT(mmp_server_destroy(s) == MMP_OK);
  EXPECT(mmp_server_destroy(nullptr) == MMP_OK);
  std::printf("abi driver: %d failures\n", fails);
  return fails ? 1 : 0;
}
