// Exercises the product's host-side parser and planner (program.cpp) under
// AddressSanitizer and UndefinedBehaviorSanitizer on accepted and rejected
// programs; checks the status each one gets.  Exit status 0 when all match.
#include <cstdio>
#include <string>

#include "../../paper_2503_21937_amd/csrc/program.h"

int main() {
  struct Case {
    const char* text;
    int want;  // 0 accepted, 2 parse error, 3 unsupported
  } cases[] = {
      {".input edge/2\npath(x, y) :- edge(x, y).\npath(x, z) :- edge(x, y), path(y, z).\n", 0},
      {".input edge/2\nsg(x, y) :- edge(p, x), edge(p, y), x != y.\nsg(x, y) :- edge(a, x), sg(a, b), edge(b, y).\n", 0},
      {".input e/2\nwalk(x, y, 1) :- e(x, y).\nwalk(x, z, d + 1) :- walk(x, y, d), e(y, z), d < 4.\n", 0},
      {".input e/2\nq(x, (y * 3 + 1) % 7, y / 2) :- e(x, y), x <= y, x >= 1, y == 2 * x.\n", 0},
      {".input e/2\nany() :- e(x, y), x != y.\nloop(x) :- e(x, x).\nc(x, z) :- e(x, 3), e(3, z).\n", 0},
      {".input a/2\n.input s/2\n.input l/2\n.input t/2\npt(v, o) :- a(v, o).\npt(v, o) :- s(v, w), pt(w, o).\n"
       "pt(v, o) :- l(v, p), pt(p, q), pt(q, o).\npt(q, o) :- t(p, w), pt(p, q), pt(w, o).\n", 0},
      {"path(x, y) :- edge(x, y", 2},
      {"p(x) :- e(x, y), x <> y.", 2},
      {"p(x) :- e(x, y), z > 1.", 3},
      {"p(x, w + 1) :- e(x, y).", 3},
      {"p(x) :- x > 1.", 3},
      {"p(a) :- q(a), r(b).", 3},
      {"p(a) :- q(a, b), r(b, c), s(c, d), t(d, a).", 3},
      {".input edge/2\nedge(x, y) :- edge(y, x).", 3},
      {".input e/5\n", 3},
      {"", 2},
  };
  int bad = 0;
  for (const Case& c : cases) {
    for (int frozen = 0; frozen < 2; ++frozen) {
      dlfix::Program p;
      std::string err;
      const int rc = dlfix::parse_and_plan(c.text, frozen != 0, false, p, err);
      if (rc != c.want) {
        std::fprintf(stderr, "status %d (want %d) for: %s\n  %s\n", rc, c.want, c.text, err.c_str());
        ++bad;
      }
    }
  }
  if (bad) return 1;
  std::printf("planner driver ok\n");
  return 0;
}
