// Host-side grid object: owns device buffers of one simulation and drives
// the stage/controller kernels on its stream.
#pragma once

#include <memory>
#include <vector>

#include "common.h"
#include "demag.h"
#include "elastic.h"
#include "field.h"
#include "prof.h"

namespace mmp {

struct GridBase {
  int nx, ny, nz;
  double d[3];
  long N;
  int precision = -1;
  int nsub = 1;
  bool params_set = false;
  bool state_set = false;
  hipStream_t own_stream = nullptr;
  hipStream_t stream = nullptr;
  Prof prof;
  mmp_params p{};
  std::vector<uint16_t> grain;
  std::vector<double> grain_axes;
  virtual ~GridBase() {}
  virtual int apply_params() = 0;
  virtual int set_state(const double* m, const double* u, const double* v, double t) = 0;
  virtual int get_state(double* m, double* u, double* v, double* t, double* dt) = 0;
  virtual int eval(uint32_t mask, double* b, double* e) = 0;
  virtual int step(double dt_fixed, mmp_step_info* info) = 0;
  virtual int run_fixed(double dt, long long n, mmp_step_info* info) = 0;
  virtual int run(double t_end, const mmp_run_opts* o, mmp_run_info* info) = 0;
  virtual long long bytes() const = 0;
  virtual int tensor(double* n6) = 0;
  virtual int get_plan(mmp_plan* out) = 0;
  virtual int set_plan(const mmp_plan* in) = 0;
  virtual int autotune(mmp_plan* out) = 0;
  virtual int set_graphs(bool on) = 0;
  // non-blocking adaptive run used by the server: begin, enqueue chunks of
  // attempts (each followed by an async controller read-back and an event;
  // at most two in flight), poll the oldest for completion
  virtual int run_begin(double t_end) = 0;
  virtual int run_chunk(int attempts) = 0;
  virtual int run_poll(bool* finished, int* status, long long* steps, long long* rejects) = 0;
  virtual int chunks_in_flight() const = 0;
};

GridBase* make_grid(int precision);

}  // namespace mmp

struct mmp_grid_s {
  int nx, ny, nz;
  double d[3];
  std::unique_ptr<mmp::GridBase> impl;
  hipStream_t user_stream = nullptr;
};
