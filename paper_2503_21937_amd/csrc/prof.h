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
  // Elapsed times and bytes of records into per-family totals k[fam]
  // (launches, ms, bytes).
  template <typename Timing>
  static void fold(const std::vector<Rec>& rs, Timing* k) {
    for (const Rec& r : rs) {
      float ms = 0.0f;
      if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) {
        (void)hipGetLastError();  // do not leave the error for the next caller
        continue;
      }
      k[r.fam].launches += 1;
      k[r.fam].ms += ms;
      k[r.fam].bytes += r.bytes;
    }
  }
  // Records launched together inside a graph, timed as one span of `ms`
  // by events around the graph launch: every record counts as a launch and
  // adds its bytes; the span's time goes to the first record's family (the
  // graphs timed this way hold one family).
  template <typename Timing>
  static void fold_span(const std::vector<Rec>& rs, float ms, Timing* k) {
    if (rs.empty()) return;
    for (const Rec& r : rs) {
      k[r.fam].launches += 1;
      k[r.fam].bytes += r.bytes;
    }
    k[rs.front().fam].ms += ms;
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
