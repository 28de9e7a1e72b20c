// Per-kernel-class timing with HIP events on the launching stream.
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

namespace mmp {

enum ProfId {
  P_FFTX_FWD = 0,
  P_FFTY_FWD,
  P_FFTZ_MUL,
  P_FFTY_INV,
  P_FFTX_INV,
  P_FFTY_MUL2D,
  P_FIELD,
  P_COMBINE,
  P_CONTROL,
  P_ELASTIC,
  P_REDUCE,
  P_COUNT
};

extern const char* const kProfNames[P_COUNT];

// Events are recorded around launches while enabled and resolved lazily, so
// timing adds no host synchronisation inside the timed region.
struct Prof {
  bool on = false;
  hipStream_t st = nullptr;
  struct Pending { int id; hipEvent_t a, b; };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> pool;
  double total_ms[P_COUNT] = {};
  long long count[P_COUNT] = {};

  hipEvent_t get();
  void begin(int id, hipStream_t s, hipEvent_t* a);
  void end(int id, hipStream_t s, hipEvent_t a);
  void resolve();
  void reset();
  ~Prof();
};

struct ProfScope {
  Prof* p;
  int id;
  hipStream_t s;
  hipEvent_t a = nullptr;
  ProfScope(Prof* p_, int id_, hipStream_t s_) : p(p_), id(id_), s(s_) {
    if (p && p->on) p->begin(id, s, &a);
  }
  ~ProfScope() {
    if (p && p->on) p->end(id, s, a);
  }
};

}  // namespace mmp
