// Request server: continuous batching of relaxation solves on one GPU.
//
// Requests arrive on any thread (mmp_submit) and wait in a FIFO queue.  A
// worker thread admits the queue head whenever a slot is free and its
// device footprint fits the remaining HBM budget; a builder thread then
// sets its grid up (own stream, own FP64 demag tensor and spectrum, first
// stage) while the worker keeps the running requests going.  Requests that
// can share one stage sequence (Dormand-Prince, no elasticity; with or
// without demag) join a batch per sublattice count: every stage of all
// members is one launch per demag pass and one field launch over device
// work tables, 8 attempts per captured graph.  The others get chunks of
// attempts on their own streams, round robin, so the kernels of different
// requests overlap on the device.  Every request keeps its own device-side
// step control and runs the arithmetic it would run alone, so its result
// does not depend on what else is in flight.  A request that finishes is
// reduced on the device (average m per sublattice, total energy), its
// memory returned, and the next queued request admitted.  Results are read
// with mmp_poll.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <string>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "grid.h"

using namespace mmp;

namespace {

struct Req {
  uint64_t ticket;
  mmp_request r;
  std::vector<double> m0;
  std::vector<uint16_t> grain;
  std::vector<double> gaxes;
  double t_submit;
  double t_admit = 0;
  int64_t footprint = 0;
  mmp_grid g = nullptr;
  int chunk = 8;
  bool try_batch = false;
  bool batched = false;
  int setup_rc = 0;
  std::string err;   // message of the call that failed the request
};

// Device footprint of a request: the buffers Grid<T>::alloc_layout makes
// for its parameters (state pair, stage pair, 7 slopes; with elasticity u
// and v pairs, their stage pairs, 14 slopes and the strain, strain-rate and
// stress tensors; grain ids and axes; the demag spectra, kernel and field),
// the transient FP64 tensor of the demag build, and 1 MiB of small buffers.
int64_t estimate_bytes(const mmp_request& r, int precision) {
  const int64_t N = (int64_t)r.nx * r.ny * r.nz;
  const int64_t rb = precision == MMP_FP64 ? 8 : 4;
  const int ns = r.params.nsub;
  int64_t b = (4 + 7) * (int64_t)ns * 3 * N * rb;  // state, stages, k
  if (r.params.elastic) b += (8 * 3 + 14 * 3 + 3 * 6) * N * rb;
  if (r.params.ngrains > 0) b += N * 2 + (int64_t)r.params.ngrains * 3 * rb;
  if (r.params.demag) {
    DemagPlan p;
    if (demag_plan(r.nx, r.ny, r.nz, (int)rb, nullptr, &p, r.params.pbc) == 0)
      b += (int64_t)(p.s1_elems + p.s2_elems) * 2 * rb + (int64_t)p.k_elems * rb + 3 * N * rb +
           6 * N * 8 /* FP64 tensor during the build */ +
           (int64_t)6 * r.nz * (r.ny + p.Hy) * p.Hx * 8;
  }
  return b + (1 << 20);
}

}  // namespace

// Attempts per chunk for `cells` cell-sublattices: about 2^23 / (cells +
// 2^15), between 8 and 128, i.e. a few ms of device work whether the grid is
// large (time per attempt grows with its cells) or small (an attempt still
// costs some tens of us of launches and latency).
static int chunk_attempts(long long cells) {
  return (int)std::max<long long>(8, std::min<long long>(128, (1LL << 23) / (cells + (1LL << 15))));
}

struct mmp_server_s {
  mmp_server_opts o{};
  std::mutex mu;
  std::condition_variable cv;
  std::deque<Req*> queue;       // submitted, waiting for admission
  std::deque<Req*> to_build;    // admitted, grid not yet set up
  std::deque<Req*> built;       // set up, not yet placed by the worker
  int building = 0;             // admitted and not yet placed
  std::condition_variable bcv;  // wakes the builder
  std::thread builder;
  std::vector<Req*> active;
  std::map<uint64_t, mmp_result> done;
  std::map<uint64_t, int> known;
  std::atomic<bool> stop{false};
  uint64_t next_ticket = 1;
  int64_t used = 0;
  std::thread worker;
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
  // grids without demag step together in one batch per sublattice count
  struct BatchState {
    BatchBase* b = nullptr;
    std::vector<Req*> members, joining;
    bool draining = false;
  };
  BatchState batches[2];

  ~mmp_server_s() {
    for (auto& B : batches) delete B.b;
  }

  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }

  void finish(Req* q, int status) {
    if (status < 0 && q->err.empty()) q->err = mmp_last_error();
    if (status < 0 && std::getenv("MMP_SERVER_LOG"))
      std::fprintf(stderr, "mmp server: request %llu failed (%d): %s\n",
                   (unsigned long long)q->ticket, status, q->err.c_str());
    mmp_result res{};
    res.status = status;
    res.nsub = q->r.params.nsub;
    res.t_submit = q->t_submit;
    res.t_admit = q->t_admit;
    if (q->g && q->g->impl && status == MMP_OK) {
      // averages and energies reduced on the device: 19 doubles come back,
      // not the state
      double avg[9] = {}, e[MMP_NENERGY] = {};
      const int rc = q->g->impl->summary(avg, e);
      if (rc == MMP_OK) {
        for (int s = 0; s < res.nsub; ++s)
          for (int c = 0; c < 3; ++c) res.m_avg[s][c] = avg[s * 3 + c];
        double et = 0;
        for (int k = 0; k < MMP_NENERGY; ++k) et += e[k];
        res.energy = et;
      } else {
        res.status = rc;
      }
      // the stream is idle after the summary: drain the chunks in flight
      long long steps = 0, rejects = 0;
      bool fin = false;
      int st = 0;
      if (q->g->impl)
        do {
          if (q->g->impl->run_poll(&fin, &st, &steps, &rejects) != 0) break;
        } while (q->g->impl->chunks_in_flight() > 0);
      res.steps = steps;
      res.rejects = rejects;
    }
    if (q->g) mmp_grid_destroy(q->g);
    q->g = nullptr;
    res.t_done = now();
    std::lock_guard<std::mutex> lk(mu);
    used -= q->footprint;
    done[q->ticket] = res;
    delete q;
  }

  // Builder thread: creates an admitted request's grid (parameters, demag
  // tensor and spectrum, state, first stage) on the grid's own stream while
  // the worker keeps the running requests' chunks flowing.
  int setup_request(Req* q) {
    // the set-up allocates and copies synchronously: it must not overlap a
    // graph capture on the worker thread
    DeviceLock lk(device_mutex());
    mmp_grid g = nullptr;
    int rc = mmp_grid_create(q->r.nx, q->r.ny, q->r.nz, q->r.cellsize, &g);
    if (rc) return rc;
    q->g = g;
    mmp_params p = q->r.params;
    p.struct_size = sizeof(mmp_params);
    p.precision = o.precision;
    p.grain = q->grain.empty() ? nullptr : q->grain.data();
    p.grain_axes = q->gaxes.empty() ? nullptr : q->gaxes.data();
    if ((rc = mmp_set_params(g, &p))) return rc;
    q->try_batch = o.batch && !p.elastic && (p.nsub == 1 || p.nsub == 2);
    if (q->try_batch && p.demag) {
      // the batch runs every demag pass through the LDS kernels: the
      // request's own first stage (and its final energy) uses them too, so
      // its result does not depend on whether it was batched
      mmp_plan pl{};
      pl.struct_size = sizeof(pl);
      if (mmp_get_plan(g, &pl) == MMP_OK) {
        pl.lds_axes = 7;
        (void)mmp_set_plan(g, &pl);
      }
    }
    if ((rc = mmp_set_state(g, q->m0.data(), nullptr, nullptr, 0.0))) return rc;
    return g->impl->run_begin(q->r.t_relax);
  }

  void builder_loop() {
    while (true) {
      Req* q = nullptr;
      {
        std::unique_lock<std::mutex> lk(mu);
        bcv.wait(lk, [&] { return stop.load() || !to_build.empty(); });
        if (stop.load()) return;   // the rest is finished at shutdown
        q = to_build.front();
        to_build.pop_front();
      }
      q->setup_rc = setup_request(q);
      if (q->setup_rc) q->err = std::string("set-up: ") + mmp_last_error();
      {
        std::lock_guard<std::mutex> lk(mu);
        built.push_back(q);
      }
      cv.notify_all();
    }
  }

  // Worker: a set-up request joins its batch or starts its own chunks.
  int place_request(Req* q) {
    if (q->try_batch) {
      const int ns = q->r.params.nsub;
      BatchState& B = batches[ns - 1];
      if (!B.b) B.b = make_batch(o.precision, ns);
      if (B.b->accepts(q->g->impl.get())) {
        q->batched = true;
        B.joining.push_back(q);
        B.draining = true;
        return 0;
      }
    }
    // attempts per chunk: a few ms of device work for any grid size (an
    // attempt costs some tens of us of launches and latency on top of its
    // cells); two chunks stay in flight so the device never waits for the
    // host
    const int64_t N = (int64_t)q->r.nx * q->r.ny * q->r.nz * q->r.params.nsub;
    q->chunk = chunk_attempts(N);
    if (int rc = q->g->impl->run_chunk(q->chunk)) return rc;
    return q->g->impl->run_chunk(q->chunk);
  }

  static bool member_done(Req* q, int* status) {
    bool fin = false;
    int st = 0;
    long long steps = 0, rejects = 0;
    const int rc = q->g->impl->run_poll(&fin, &st, &steps, &rejects);
    *status = rc != 0 ? rc : st;
    return rc != 0 || fin;
  }

  // a failed chunk or poll: the batch drops its members and chunks (after
  // its stream has drained, so no kernel still reads their grids), every
  // member and every request waiting to join is finished with the error,
  // and the next batched request starts a fresh batch
  void fail_batch(BatchState& B, int rc) {
    B.b->abandon();
    for (Req* q : B.members) finish(q, rc);
    for (Req* q : B.joining) finish(q, rc);
    B.members.clear();
    B.joining.clear();
    B.draining = false;
    delete B.b;
    B.b = nullptr;
  }

  // one round of a batch: collect finished chunks; when it is idle and a
  // member has finished or requests wait to join, change the membership;
  // keep two chunks in flight otherwise.  Returns whether anything moved.
  bool step_batch(BatchState& B) {
    if (!B.b) return false;
    bool any = false;
    while (B.b->in_flight() > 0) {
      const int rc = B.b->poll();
      if (rc == MMP_PENDING) break;
      any = true;
      if (rc != 0) {
        fail_batch(B, rc);
        return true;
      }
      int st = 0;
      for (Req* q : B.members)
        if (member_done(q, &st)) B.draining = true;
    }
    // membership changes wait until the batch is idle; otherwise the next
    // chunk goes out as soon as one has finished, so the device always has
    // one queued behind the one it runs
    const bool change = B.draining || !B.joining.empty();
    if (change && B.b->in_flight() > 0) return any;
    if (change) {
      for (size_t i = 0; i < B.members.size();) {
        Req* q = B.members[i];
        int st = 0;
        if (member_done(q, &st)) {
          (void)B.b->remove(q->g->impl.get());
          B.members.erase(B.members.begin() + i);
          finish(q, st);
        } else {
          ++i;
        }
      }
      for (Req* q : B.joining) {
        const int rc = B.b->add(q->g->impl.get());
        if (rc) finish(q, rc);
        else B.members.push_back(q);
      }
      B.joining.clear();
      B.draining = false;
      any = true;
    }
    if (!B.members.empty()) {
      const int chunk = chunk_attempts(std::max<long long>(1, B.b->cells()));
      while (B.b->in_flight() < 2) {
        const int rc = B.b->run_chunk(chunk);
        if (rc) {
          fail_batch(B, rc);
          return true;
        }
        any = true;
      }
    }
    return any;
  }

  // requests admitted but not yet placed, at shutdown
  void finish_unplaced() {
    std::vector<Req*> left;
    {
      std::lock_guard<std::mutex> lk(mu);
      left.assign(to_build.begin(), to_build.end());
      left.insert(left.end(), built.begin(), built.end());
      to_build.clear();
      built.clear();
      building = 0;
    }
    for (Req* q : left) finish(q, MMP_E_STATE);
  }

  int batched_count() const {
    return (int)(batches[0].members.size() + batches[0].joining.size() +
                 batches[1].members.size() + batches[1].joining.size());
  }

  void loop() {
    while (!stop.load()) {
      // admission: the queue head goes to the builder once a slot is free
      // and its footprint fits the budget (or nothing else runs)
      {
        std::lock_guard<std::mutex> lk(mu);
        while (!queue.empty()) {
          const int busy = (int)active.size() + batched_count() + building;
          if (busy >= o.max_active) break;
          Req* h = queue.front();
          if (used + h->footprint > o.hbm_budget && busy > 0) break;
          queue.pop_front();
          used += h->footprint;
          h->t_admit = now();
          to_build.push_back(h);
          ++building;
        }
      }
      bcv.notify_one();
      // requests the builder has set up join their batch or start chunks
      bool any = false;
      {
        std::vector<Req*> ready;
        {
          std::lock_guard<std::mutex> lk(mu);
          ready.assign(built.begin(), built.end());
          built.clear();
        }
        for (Req* q : ready) {
          any = true;
          const int rc = q->setup_rc ? q->setup_rc : place_request(q);
          {
            std::lock_guard<std::mutex> lk(mu);
            --building;
          }
          if (rc) finish(q, rc);
          else if (!q->batched) active.push_back(q);
        }
      }
      // progress
      for (auto& B : batches) any |= step_batch(B);
      for (size_t i = 0; i < active.size();) {
        Req* q = active[i];
        bool fin = false;
        int st = 0;
        long long steps = 0, rejects = 0;
        const int rc = q->g->impl->run_poll(&fin, &st, &steps, &rejects);
        if (rc == MMP_PENDING) { ++i; continue; }
        any = true;
        if (rc != 0 || fin) {
          active.erase(active.begin() + i);
          finish(q, rc != 0 ? rc : st);
          continue;
        }
        const int rc2 = q->g->impl->run_chunk(q->chunk);
        if (rc2 != 0) {
          active.erase(active.begin() + i);
          finish(q, rc2);
          continue;
        }
        ++i;
      }
      if (!any) {
        std::unique_lock<std::mutex> lk(mu);
        cv.wait_for(lk, std::chrono::microseconds(50));
      }
    }
    for (Req* q : active) finish(q, MMP_E_STATE);
    active.clear();
    for (auto& B : batches) {
      if (B.b) {
        while (B.b->in_flight() > 0 && B.b->poll() == MMP_PENDING) {
        }
      }
      for (Req* q : B.members) finish(q, MMP_E_STATE);
      for (Req* q : B.joining) finish(q, MMP_E_STATE);
      B.members.clear();
      B.joining.clear();
    }
  }
};

extern "C" {

mmp_status mmp_server_create(const mmp_server_opts* o, mmp_server* out) {
  try {
    if (!o || !out || o->struct_size != sizeof(mmp_server_opts)) {
      set_error("bad server options");
      return MMP_E_ARG;
    }
    if (o->hbm_budget <= 0 || o->max_active < 1 ||
        (o->precision != MMP_FP32 && o->precision != MMP_FP64)) {
      set_error("bad server options");
      return MMP_E_ARG;
    }
    mmp_server s = new mmp_server_s();
    s->o = *o;
    s->worker = std::thread([s] { s->loop(); });
    s->builder = std::thread([s] { s->builder_loop(); });
    *out = s;
    return MMP_OK;
  } catch (...) {
    set_error("server creation failed");
    return MMP_E_NOMEM;
  }
}

mmp_status mmp_submit(mmp_server s, const mmp_request* r, uint64_t* ticket) {
  try {
    if (!s || !r || !ticket || r->struct_size != sizeof(mmp_request)) {
      set_error("bad request");
      return MMP_E_ARG;
    }
    if (r->nx < 1 || r->ny < 1 || r->nz < 1 || !r->m0 || !(r->t_relax > 0) ||
        r->params.nsub < 1 || r->params.nsub > 3) {
      set_error("bad request");
      return MMP_E_ARG;
    }
    const int64_t N = (int64_t)r->nx * r->ny * r->nz;
    Req* q = new Req();
    q->r = *r;
    q->m0.assign(r->m0, r->m0 + (size_t)r->params.nsub * 3 * N);
    q->r.m0 = nullptr;
    if (r->params.ngrains > 0 && r->params.grain && r->params.grain_axes) {
      q->grain.assign(r->params.grain, r->params.grain + N);
      q->gaxes.assign(r->params.grain_axes, r->params.grain_axes + 3 * r->params.ngrains);
    }
    q->footprint = estimate_bytes(*r, s->o.precision);
    if (q->footprint > s->o.hbm_budget) {
      delete q;
      set_error("request exceeds the HBM budget");
      return MMP_E_TOO_LARGE;
    }
    std::lock_guard<std::mutex> lk(s->mu);
    q->ticket = s->next_ticket++;
    q->t_submit = s->now();
    s->known[q->ticket] = 1;
    s->queue.push_back(q);
    *ticket = q->ticket;
    s->cv.notify_all();
    return MMP_OK;
  } catch (...) {
    set_error("submit failed");
    return MMP_E_NOMEM;
  }
}

mmp_status mmp_poll(mmp_server s, uint64_t ticket, mmp_result* out) {
  if (!s || !out) { set_error("bad argument"); return MMP_E_ARG; }
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->done.find(ticket);
  if (it != s->done.end()) {
    // a result is handed out once; the server keeps nothing of a request
    // after that, so a long stream does not grow its tables
    *out = it->second;
    s->done.erase(it);
    s->known.erase(ticket);
    return MMP_OK;
  }
  if (s->known.count(ticket)) return MMP_PENDING;
  set_error("unknown ticket");
  return MMP_E_TICKET;
}

mmp_status mmp_server_destroy(mmp_server s) {
  if (!s) return MMP_OK;
  s->stop.store(true);
  s->cv.notify_all();
  s->bcv.notify_all();
  if (s->worker.joinable()) s->worker.join();
  if (s->builder.joinable()) s->builder.join();
  s->finish_unplaced();
  for (Req* q : s->queue) delete q;
  delete s;
  return MMP_OK;
}

double mmp_server_clock(mmp_server s) { return s ? s->now() : 0.0; }

}  // extern "C"
