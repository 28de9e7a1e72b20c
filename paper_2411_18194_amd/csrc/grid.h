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
  // device-pointer variants: FP64 device buffers in the host layouts,
  // enqueued on the grid's stream, no host synchronisation
  virtual int set_state_device(const double* m, const double* u, const double* v, double t) = 0;
  virtual int get_state_device(double* m, double* u, double* v, double* t_dt) = 0;
  virtual int eval_device(uint32_t mask, double* b) = 0;
  virtual int step(double dt_fixed, mmp_step_info* info) = 0;
  virtual int run_fixed(double dt, long long n, mmp_step_info* info) = 0;
  virtual int run(double t_end, const mmp_run_opts* o, mmp_run_info* info) = 0;
  virtual long long bytes() const = 0;
  virtual int tensor(double* n6) = 0;
  virtual int stray(double height, double* out) = 0;
  virtual int stray_noalloc(double height, double* out_dev) = 0;
  // averages of m per sublattice (m_avg[3 nsub], reduced on the device in
  // FP64) and the per-term energies (e[MMP_NENERGY]) of the current state;
  // synchronous
  virtual int summary(double* m_avg, double* e) = 0;
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
  // for a batch: the member's stream is idle and its last controller state
  // is `c` (host copy)
  virtual void set_chunk_state(const void* c) = 0;
};

GridBase* make_grid(int precision);

// Many grids stepped together: each stage of every member is one launch
// (a device work table of (grid, block)), the step controllers and stage-2
// combinations one launch each, 8 attempts per captured HIP graph, on the
// batch's own stream.  Members keep their own buffers and device-side step
// control, so each one takes exactly the steps it would take alone.  Only
// grids without demag and elasticity join, all with the batch's precision
// and sublattice count, and membership changes only while no chunk is in
// flight (kernels of a chunk read every member's controller).
struct BatchBase {
  virtual ~BatchBase() {}
  virtual bool accepts(const GridBase* g) const = 0;
  // g must have begun its run (run_begin) on its own stream
  virtual int add(GridBase* g) = 0;
  virtual int remove(GridBase* g) = 0;
  virtual int size() const = 0;
  virtual int in_flight() const = 0;
  // enqueue `attempts` attempts of every member, then a read-back of their
  // controllers (at most two chunks in flight)
  virtual int run_chunk(int attempts) = 0;
  // MMP_PENDING while the oldest chunk runs; else its controller states are
  // handed to the members (their run_poll reports them)
  virtual int poll() = 0;
  virtual long long cells() const = 0;
  // after a failed chunk or poll: wait for the batch's stream, drop every
  // member and every chunk in flight; the batch is then empty and idle
  virtual void abandon() = 0;
};

BatchBase* make_batch(int precision, int nsub);

}  // namespace mmp

struct mmp_grid_s {
  int nx, ny, nz;
  double d[3];
  std::unique_ptr<mmp::GridBase> impl;
  hipStream_t user_stream = nullptr;
};
