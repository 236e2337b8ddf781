// Exercises the CPU oracle (oracle/) under AddressSanitizer and
// UndefinedBehaviorSanitizer: every semiring, expressions, batching, top-k,
// reverse mode, the transitive-closure column solver and the worklist
// points-to solver, on small seeded inputs.  Exit status 0 when every call
// succeeds; the sanitizers abort on the first error they find.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "../../oracle/dlref.h"

static void check(int rc, const char* what) {
  if (rc) {
    std::fprintf(stderr, "%s failed (%d)\n", what, rc);
    std::exit(1);
  }
}

static void run_program(const char* prog, int sr, int batched, const char* in, const char* out, int arity,
                        unsigned seed, bool backward) {
  ref_engine* e = nullptr;
  char err[256];
  check(ref_create(prog, sr, 3, batched, &e, err, sizeof err), err);
  std::mt19937 rng(seed);
  const size_t n = 120;
  std::vector<uint32_t> cols(n * arity), samp(n);
  std::vector<float> tags(n);
  for (size_t i = 0; i < n; ++i) {
    for (int c = 0; c < arity; ++c) cols[i * arity + c] = rng() % 30;
    samp[i] = batched ? (uint32_t)(i % 3) : 0u;
    tags[i] = 0.1f + 0.8f * (float)(rng() % 1000) / 1000.0f;
  }
  size_t m = n;
  if (sr == REF_TOPK || sr == REF_DIFF_TOPK) m = batched ? 150 : 50;  // <= 64 facts per sample
  if (m > n) m = n;
  check(ref_add_facts(e, in, m, batched ? samp.data() : nullptr, cols.data(), sr == REF_BOOL ? nullptr : tags.data()),
        "add_facts");
  check(ref_run(e), "run");
  const long k = ref_size(e, out);
  std::vector<uint32_t> os(k + 1), oc((k + 1) * 4);
  std::vector<double> val(k + 1), prob(k + 1);
  std::vector<int32_t> cnt(k + 1), rf(k + 1);
  std::vector<uint64_t> bits((k + 1) * 3);
  std::vector<float> p((k + 1) * 3);
  check(ref_read(e, out, os.data(), oc.data(), val.data(), cnt.data(), bits.data(), p.data(), prob.data(), rf.data()),
        "read");
  if (backward) {
    std::vector<double> g(k + 1, 1.0), gi(m + 1);
    check(ref_backward(e, out, g.data()), "backward");
    check(ref_read_grad(e, in, gi.data()), "read_grad");
  }
  ref_free(e);
}

int main() {
  const char* tc = ".input edge/2\npath(x, y) :- edge(x, y).\npath(x, z) :- edge(x, y), path(y, z).\n";
  const char* sg = ".input edge/2\nsg(x, y) :- edge(p, x), edge(p, y), x != y.\n"
                   "sg(x, y) :- edge(a, x), sg(a, b), edge(b, y).\n";
  const char* walk = ".input edge/2\nwalk(x, y, 1) :- edge(x, y).\n"
                     "walk(x, z, d + 1) :- walk(x, y, d), edge(y, z), d < 4.\n"
                     "q(x, y / (x + 1), y % 7) :- edge(x, y), x <= y.\nany() :- edge(x, x).\n";
  for (int sr = REF_BOOL; sr <= REF_DIFF_TOPK; ++sr) {
    const bool diff = sr == REF_DIFF_ADDMULT || sr == REF_DIFF_TOPK;
    run_program(tc, sr, 0, "edge", "path", 2, 1 + sr, diff);
    run_program(tc, sr, 1, "edge", "path", 2, 11 + sr, diff);
    if (sr != REF_DIFF_ADDMULT) run_program(sg, sr, 0, "edge", "sg", 2, 21 + sr, false);
    run_program(walk, sr, 0, "edge", "walk", 2, 31 + sr, false);
  }
  // column solver and worklist solver
  std::mt19937 rng(7);
  std::vector<uint32_t> src(200), dst(200);
  std::vector<float> w(200);
  for (int i = 0; i < 200; ++i) {
    src[i] = rng() % 60;
    dst[i] = rng() % 60;
    w[i] = 0.5f;
  }
  std::vector<uint8_t> pres(60);
  std::vector<double> tag(60), gcol(60, 1.0), gedge(200);
  std::vector<int32_t> found(60);
  int32_t rounds = 0;
  for (int sr = REF_BOOL; sr <= REF_ADDMULT; ++sr)
    check(ref_tc_column(60, 200, src.data(), dst.data(), w.data(), sr, 5, pres.data(), tag.data(), found.data(),
                        &rounds, sr == REF_ADDMULT ? gcol.data() : nullptr, sr == REF_ADDMULT ? gedge.data() : nullptr),
          "tc_column");
  std::vector<uint32_t> addr(2 * 40), rel(2 * 150);
  for (auto& x : addr) x = rng() % 80;
  for (auto& x : rel) x = rng() % 80;
  ref_pts* pts = ref_andersen(80, 40, addr.data(), 150, rel.data(), 60, rel.data(), 50, rel.data() + 100);
  const long np = ref_pts_size(pts);
  std::vector<uint32_t> pv(np + 1), po(np + 1);
  ref_pts_read(pts, pv.data(), po.data());
  ref_pts_free(pts);
  std::printf("oracle driver ok\n");
  return 0;
}
