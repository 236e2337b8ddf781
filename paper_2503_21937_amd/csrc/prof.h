// Optional per-kernel timing with HIP events on the launching stream.  When
// an engine enables it, launchers bracket their kernel with two events and
// add the kernel's algorithmic bytes (what the operation must read and write
// at minimum); the engine sums the elapsed times after the run.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

namespace dlfix {

struct Profiler {
  struct Rec {
    hipEvent_t a, b;
    int fam;
    double bytes;
  };
  uint32_t mask = 0;
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  // Launches whose unit count only the device knows add `deferred_per`
  // bytes per unit to family `deferred_fam`; the engine supplies the run's
  // total of those units afterwards (it accumulates them on the device).
  int deferred_fam = -1;
  double deferred_per = 0.0;
  hipEvent_t get() {
    if (used == pool.size()) {
      hipEvent_t ev;
      if (hipEventCreate(&ev) != hipSuccess) return nullptr;
      pool.push_back(ev);
    }
    return pool[used++];
  }
  void begin(int fam, hipStream_t st) {
    if (!(mask >> fam & 1u)) return;
    Rec r{get(), get(), fam, 0.0};
    if (r.a && r.b) {
      (void)hipEventRecord(r.a, st);
      recs.push_back(r);
    }
  }
  void end(int fam, hipStream_t st, double bytes) {
    if (!(mask >> fam & 1u) || recs.empty() || recs.back().fam != fam) return;
    recs.back().bytes = bytes;
    (void)hipEventRecord(recs.back().b, st);
  }
  void defer(int fam, double per_unit) {
    if (!(mask >> fam & 1u)) return;
    deferred_fam = fam;
    deferred_per = per_unit;
  }
  ~Profiler() {
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
  }
};

extern thread_local Profiler* g_prof;

}  // namespace dlfix

#define DL_PROF_BEGIN(fam, st) \
  do {                          \
    if (::dlfix::g_prof) ::dlfix::g_prof->begin((fam), (st)); \
  } while (0)
#define DL_PROF_END(fam, st, bytes) \
  do {                               \
    if (::dlfix::g_prof) ::dlfix::g_prof->end((fam), (st), (double)(bytes)); \
  } while (0)
#define DL_PROF_DEFER(fam, per_unit) \
  do {                                \
    if (::dlfix::g_prof) ::dlfix::g_prof->defer((fam), (double)(per_unit)); \
  } while (0)
