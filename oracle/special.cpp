// CPU oracle, special-purpose solvers -- TEST INFRASTRUCTURE ONLY.
//
// ref_tc_column: the naive Jacobi rounds of the transitive-closure program
// restricted to one target column.  In
//     path(x, y) :- edge(x, y).
//     path(x, z) :- edge(x, y), path(y, z).
// every derivation of path(x, z) reads only path(y, z) with the same z, so a
// column evolves on its own, round for round, exactly as inside the full
// evaluation (same derivations, same discovery rounds, same +-order: the base
// rule's derivation first, then the recursive rule's in ascending y).  It lets
// tests check sampled columns of graphs too large for the generic evaluator.
//
// ref_andersen: textbook worklist solver (difference propagation over a
// dynamically growing subset graph) for the least solution of the four
// points-to rules; a pin for the boolean fixpoint that does not use rounds.
#include "dlref.h"

#include <algorithm>
#include <cmath>
#include <limits>
#include <numeric>
#include <unordered_set>
#include <vector>

extern "C" {

int ref_tc_column(int n, size_t m, const uint32_t* src, const uint32_t* dst, const float* w, int semiring,
                  uint32_t z, uint8_t* present, double* tag, int32_t* found, int32_t* rounds,
                  const double* grad_col, double* grad_edge) {
  if (semiring < REF_BOOL || semiring > REF_DIFF_ADDMULT || z >= (uint32_t)n) return 1;
  const bool frozen = semiring == REF_ADDMULT || semiring == REF_DIFF_ADDMULT;
  std::vector<size_t> order(m);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) {
    if (src[a] != src[b]) return src[a] < src[b];
    return dst[a] < dst[b];
  });
  const double inf = std::numeric_limits<double>::infinity();
  auto wt = [&](size_t e) { return semiring == REF_BOOL ? 1.0 : (double)w[e]; };
  auto otimes = [&](double a, double b) {
    switch (semiring) {
      case REF_MAXMIN: return std::min(a, b);
      case REF_MINPLUS: return a + b;
      case REF_BOOL: return 1.0;
      default: return a * b;
    }
  };
  auto oplus = [&](double a, double b) {
    switch (semiring) {
      case REF_MAXMIN: return std::max(a, b);
      case REF_MINPLUS: return std::min(a, b);
      case REF_BOOL: return 1.0;
      default: return std::min(1.0, a + b);
    }
  };
  std::vector<uint8_t> pres(n, 0);
  std::vector<double> t(n, semiring == REF_MINPLUS ? inf : 0.0), s(n, 0.0);
  std::vector<int32_t> fr(n, 0);
  int round = 0;
  for (round = 1;; ++round) {
    std::vector<uint8_t> any(n, 0);
    std::vector<double> c(n, 0.0), csum(n, 0.0);
    auto derive = [&](uint32_t x, double v) {
      if (frozen) {
        if (pres[x]) return;
        csum[x] += v;
      } else {
        c[x] = any[x] ? oplus(c[x], v) : v;
      }
      any[x] = 1;
    };
    for (size_t e : order)
      if (dst[e] == z) derive(src[e], wt(e));
    for (size_t e : order)
      if (pres[dst[e]]) derive(src[e], otimes(wt(e), t[dst[e]]));
    bool changed = false;
    for (int x = 0; x < n; ++x) {
      if (!any[x]) continue;
      if (frozen) {
        pres[x] = 1;
        s[x] = csum[x];
        t[x] = std::min(1.0, csum[x]);
        fr[x] = round;
        changed = true;
      } else if (!pres[x]) {
        pres[x] = 1;
        t[x] = c[x];
        fr[x] = round;
        changed = true;
      } else {
        double t2 = oplus(t[x], c[x]);
        if (t2 != t[x]) {
          t[x] = t2;
          changed = true;
        }
      }
    }
    if (!changed) break;
  }
  for (int x = 0; x < n; ++x) {
    if (present) present[x] = pres[x];
    if (tag) tag[x] = pres[x] ? (semiring == REF_BOOL ? 1.0 : t[x]) : 0.0;
    if (found) found[x] = fr[x];
  }
  if (rounds) *rounds = round;
  if (grad_col && grad_edge) {
    if (semiring != REF_DIFF_ADDMULT && semiring != REF_ADDMULT) return 2;
    // Reverse sweep over discovery rounds: a tuple found in round r was derived
    // from tuples found in rounds < r only.
    std::vector<double> adj(grad_col, grad_col + n);
    for (int r = round; r >= 1; --r) {
      for (size_t e : order) {
        uint32_t x = src[e], y = dst[e];
        if (!pres[x] || fr[x] != r || !(s[x] < 1.0)) continue;
        double g = adj[x];
        if (y == z) grad_edge[e] += g;  // base rule: value is the edge itself
        if (pres[y] && fr[y] <= r - 1) {
          grad_edge[e] += g * t[y];
          adj[y] += g * (double)w[e];
        }
      }
    }
  }
  return 0;
}

}  // extern "C"

struct ref_pts {
  std::vector<std::vector<uint32_t>> pts;  // sorted
};

namespace {
// a := a U b (both sorted); returns the elements of b that were new, sorted.
std::vector<uint32_t> merge_new(std::vector<uint32_t>& a, const std::vector<uint32_t>& b) {
  std::vector<uint32_t> fresh;
  std::set_difference(b.begin(), b.end(), a.begin(), a.end(), std::back_inserter(fresh));
  if (!fresh.empty()) {
    std::vector<uint32_t> u;
    u.reserve(a.size() + fresh.size());
    std::merge(a.begin(), a.end(), fresh.begin(), fresh.end(), std::back_inserter(u));
    a.swap(u);
  }
  return fresh;
}
}  // namespace

extern "C" {

ref_pts* ref_andersen(uint32_t nv, size_t na, const uint32_t* addr, size_t ns, const uint32_t* assign, size_t nl,
                      const uint32_t* load, size_t nst, const uint32_t* store) {
  auto* R = new ref_pts();
  auto& pts = R->pts;
  pts.assign(nv, {});
  std::vector<std::vector<uint32_t>> delta(nv), succ(nv), loads(nv), stores(nv);
  std::unordered_set<uint64_t> edges;
  std::vector<uint32_t> work;
  std::vector<char> queued(nv, 0);
  auto push = [&](uint32_t v) {
    if (!queued[v]) {
      queued[v] = 1;
      work.push_back(v);
    }
  };
  // pts[to] must include pts[from]
  auto add_edge = [&](uint32_t from, uint32_t to) {
    if (!edges.insert((uint64_t)from << 32 | to).second) return;
    succ[from].push_back(to);
    auto fresh = merge_new(pts[to], pts[from]);
    if (!fresh.empty()) {
      std::vector<uint32_t> d2;
      std::merge(delta[to].begin(), delta[to].end(), fresh.begin(), fresh.end(), std::back_inserter(d2));
      delta[to].swap(d2);
      push(to);
    }
  };
  for (size_t i = 0; i < na; ++i) {
    uint32_t v = addr[2 * i], o = addr[2 * i + 1];
    std::vector<uint32_t> one{o};
    auto fresh = merge_new(pts[v], one);
    if (!fresh.empty()) {
      merge_new(delta[v], one);
      push(v);
    }
  }
  for (size_t i = 0; i < nl; ++i) loads[load[2 * i + 1]].push_back(load[2 * i]);     // p -> v
  for (size_t i = 0; i < nst; ++i) stores[store[2 * i]].push_back(store[2 * i + 1]);  // p -> w
  for (size_t i = 0; i < ns; ++i) add_edge(assign[2 * i + 1], assign[2 * i]);         // w -> v
  while (!work.empty()) {
    uint32_t nn = work.back();
    work.pop_back();
    queued[nn] = 0;
    std::vector<uint32_t> d;
    d.swap(delta[nn]);
    if (d.empty()) continue;
    for (uint32_t q : d) {
      for (uint32_t v : loads[nn]) add_edge(q, v);   // pt(v,o) :- load(v,nn), pt(nn,q), pt(q,o)
      for (uint32_t w : stores[nn]) add_edge(w, q);  // pt(q,o) :- store(nn,w), pt(nn,q), pt(w,o)
    }
    // iterate over a snapshot: add_edge above may have grown succ[nn]
    std::vector<uint32_t> targets = succ[nn];
    for (uint32_t s : targets) {
      auto fresh = merge_new(pts[s], d);
      if (!fresh.empty()) {
        std::vector<uint32_t> d2;
        std::merge(delta[s].begin(), delta[s].end(), fresh.begin(), fresh.end(), std::back_inserter(d2));
        delta[s].swap(d2);
        push(s);
      }
    }
  }
  return R;
}

long ref_pts_size(ref_pts* R) {
  long n = 0;
  for (auto& p : R->pts) n += (long)p.size();
  return n;
}

void ref_pts_read(ref_pts* R, uint32_t* v, uint32_t* o) {
  size_t i = 0;
  for (size_t a = 0; a < R->pts.size(); ++a)
    for (uint32_t b : R->pts[a]) {
      v[i] = (uint32_t)a;
      o[i] = b;
      ++i;
    }
}

void ref_pts_free(ref_pts* R) { delete R; }

}  // extern "C"
