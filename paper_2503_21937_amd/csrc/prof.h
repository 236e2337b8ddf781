// Optional per-kernel timing with HIP events on the launching stream.  When
// an engine enables it, launchers bracket their kernel with two events and
// add the kernel's algorithmic bytes (what the operation must read and write
// at minimum); the engine sums the elapsed times after the run.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

namespace dlfix {

// Copies *src to *dst on the stream (a one-thread kernel; k_prims.hip).
void copy_word(const uint64_t* src, uint64_t* dst, hipStream_t st);

struct Profiler {
  struct Rec {
    hipEvent_t a, b;
    int fam;
    double bytes;
    double per_unit;  // bytes per unit of a count known only on the device
    int slot;         // its copy in `counts` (-1: none)
  };
  static constexpr int MAX_DEFERRED = 1 << 16;
  uint32_t mask = 0;
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  uint64_t* counts = nullptr;  // device copies of deferred counts
  int ncounts = 0;
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
    recs.back().per_unit = 0.0;
    recs.back().slot = -1;
    (void)hipEventRecord(recs.back().b, st);
  }
  // The last launch also moved per_unit bytes for each of *dcount units, a
  // count that only the device knows: snapshot it after the launch.
  void defer(int fam, hipStream_t st, const uint64_t* dcount, double per_unit) {
    if (!(mask >> fam & 1u) || recs.empty() || recs.back().fam != fam) return;
    if (!counts && hipMalloc((void**)&counts, MAX_DEFERRED * sizeof(uint64_t)) != hipSuccess) counts = nullptr;
    if (!counts || ncounts == MAX_DEFERRED) return;
    recs.back().per_unit = per_unit;
    recs.back().slot = ncounts;
    copy_word(dcount, counts + ncounts++, st);
  }
  // After the stream has drained: fold the deferred counts into the bytes.
  void resolve() {
    if (!ncounts) return;
    std::vector<uint64_t> h(ncounts);
    if (hipMemcpy(h.data(), counts, ncounts * sizeof(uint64_t), hipMemcpyDeviceToHost) != hipSuccess) return;
    for (Rec& r : recs)
      if (r.slot >= 0) r.bytes += r.per_unit * (double)h[r.slot];
  }
  ~Profiler() {
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
    if (counts) (void)hipFree(counts);
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
#define DL_PROF_DEFER(fam, st, dcount, per_unit) \
  do {                                            \
    if (::dlfix::g_prof) ::dlfix::g_prof->defer((fam), (st), (dcount), (double)(per_unit)); \
  } while (0)
