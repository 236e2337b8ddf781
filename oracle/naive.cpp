// CPU oracle: naive Jacobi evaluation of semiring Datalog -- TEST
// INFRASTRUCTURE ONLY (tests, smoke check, CPU baseline).  Shares no code
// with the HIP product path.  See dlref.h for the semantics it implements.
//
// Deliberately plain: relations are std::map from tuple to entry, rules are
// enumerated atom by atom in body order (nested loops, with a per-round
// lookup table on the positions already bound), floating point is binary64
// except the top-k proof probabilities, which the semiring defines in
// binary32 (they decide which proofs are kept).
//
// Pinned by tests/test_oracle_*.py against closed forms, textbook
// algorithms and brute force.  Parity unpinned in one regime: top-k on
// cyclic graphs beyond brute-force size (on DAGs, against path enumeration).
#include "dlref.h"

#include <algorithm>
#include <cctype>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <limits>
#include <map>
#include <memory>
#include <stdexcept>
#include <string>
#include <vector>

namespace {

struct Term {
  bool var;
  uint32_t v;  // variable index or constant
};
struct Atom {
  int rel;
  std::vector<Term> args;
};
// Arithmetic over u32 values (Sec. 5, expression evaluation: head terms
// computed from the bound variables, comparisons filtering derivations).
// + - * wrap modulo 2^32, / and % are unsigned; a division by zero voids the
// derivation.
struct Expr {
  enum Op { VAR, CONST, ADD, SUB, MUL, DIV, MOD } op = CONST;
  uint32_t v = 0;  // variable index or constant
  std::vector<Expr> kids;
};
enum Cmp { CMP_EQ, CMP_NE, CMP_LT, CMP_LE, CMP_GT, CMP_GE };
struct Cond {
  Cmp cmp;
  Expr a, b;
};
struct Rule {
  Atom head;
  std::vector<Expr> head_terms;  // one per head column
  std::vector<Atom> body;
  std::vector<Cond> conds;       // every one must hold for a derivation to count
  int nvars;
};
struct RelInfo {
  std::string name;
  int arity;
  bool input;
  bool idb;
  int first_seen;
};

struct Program {
  std::vector<RelInfo> rels;
  std::vector<Rule> rules;
  std::vector<std::vector<int>> strata;  // rule indices, evaluation order
  int find(const std::string& n) const {
    for (size_t i = 0; i < rels.size(); ++i)
      if (rels[i].name == n) return (int)i;
    return -1;
  }
};

// ----------------------------------------------------------------- parsing
struct Parser {
  std::string s;
  size_t i = 0;
  Program prog;
  int seen = 0;

  [[noreturn]] void fail(const std::string& m) {
    throw std::runtime_error("parse error at offset " + std::to_string(i) + ": " + m);
  }
  void skip() {
    while (i < s.size()) {
      if (std::isspace((unsigned char)s[i])) {
        ++i;
      } else if (s[i] == '#' || (s[i] == '/' && i + 1 < s.size() && s[i + 1] == '/')) {
        while (i < s.size() && s[i] != '\n') ++i;
      } else {
        break;
      }
    }
  }
  bool peek(char c) {
    skip();
    return i < s.size() && s[i] == c;
  }
  void expect(const char* t) {
    skip();
    size_t n = std::strlen(t);
    if (s.compare(i, n, t) != 0) fail(std::string("expected '") + t + "'");
    i += n;
  }
  std::string ident() {
    skip();
    size_t b = i;
    if (i < s.size() && (std::isalpha((unsigned char)s[i]) || s[i] == '_')) {
      while (i < s.size() && (std::isalnum((unsigned char)s[i]) || s[i] == '_')) ++i;
    }
    if (b == i) fail("expected identifier");
    return s.substr(b, i - b);
  }
  uint32_t number() {
    skip();
    size_t b = i;
    unsigned long long v = 0;
    while (i < s.size() && std::isdigit((unsigned char)s[i])) {
      v = v * 10 + (unsigned)(s[i] - '0');
      if (v > 0xffffffffull) fail("constant out of u32 range");
      ++i;
    }
    if (b == i) fail("expected number");
    return (uint32_t)v;
  }
  int relation(const std::string& name, int arity) {
    int r = prog.find(name);
    if (r < 0) {
      prog.rels.push_back({name, arity, false, false, seen++});
      return (int)prog.rels.size() - 1;
    }
    if (prog.rels[r].arity != arity) fail("arity mismatch for " + name);
    return r;
  }
  int var(std::map<std::string, int>& vars, const std::string& v) {
    auto it = vars.find(v);
    int id = it == vars.end() ? (int)vars.size() : it->second;
    if (it == vars.end()) vars[v] = id;
    return id;
  }
  // expr := term {(+|-) term}; term := factor {(*|/|%) factor};
  // factor := number | variable | ( expr )
  Expr factor(std::map<std::string, int>& vars) {
    skip();
    Expr x;
    if (peek('(')) {
      expect("(");
      x = expr(vars);
      expect(")");
    } else if (i < s.size() && std::isdigit((unsigned char)s[i])) {
      x.op = Expr::CONST;
      x.v = number();
    } else {
      x.op = Expr::VAR;
      x.v = (uint32_t)var(vars, ident());
    }
    return x;
  }
  Expr term(std::map<std::string, int>& vars) {
    Expr x = factor(vars);
    for (;;) {
      Expr::Op op;
      if (peek('*')) op = Expr::MUL;
      else if (peek('/') && !(i + 1 < s.size() && s[i + 1] == '/')) op = Expr::DIV;
      else if (peek('%')) op = Expr::MOD;
      else return x;
      ++i;
      Expr y;
      y.op = op;
      y.kids = {x, factor(vars)};
      x = y;
    }
  }
  Expr expr(std::map<std::string, int>& vars) {
    Expr x = term(vars);
    for (;;) {
      Expr::Op op;
      if (peek('+')) op = Expr::ADD;
      else if (peek('-')) op = Expr::SUB;
      else return x;
      ++i;
      Expr y;
      y.op = op;
      y.kids = {x, term(vars)};
      x = y;
    }
  }
  Cond comparison(std::map<std::string, int>& vars) {
    Cond c;
    c.a = expr(vars);
    skip();
    static const struct {
      const char* t;
      Cmp c;
    } ops[] = {{"==", CMP_EQ}, {"!=", CMP_NE}, {"<=", CMP_LE}, {">=", CMP_GE},
               {"<", CMP_LT},  {">", CMP_GT},  {"=", CMP_EQ}};
    bool found = false;
    for (auto& o : ops)
      if (s.compare(i, std::strlen(o.t), o.t) == 0) {
        i += std::strlen(o.t);
        c.cmp = o.c;
        found = true;
        break;
      }
    if (!found) fail("expected a comparison operator");
    c.b = expr(vars);
    return c;
  }
  // The head: a relation whose arguments are expressions over the body's
  // variables (a plain variable or constant is the common case).
  Atom head(std::map<std::string, int>& vars, std::vector<Expr>& terms) {
    std::string name = ident();
    expect("(");
    std::vector<Term> args;
    if (!peek(')')) {
      for (;;) {
        Expr x = expr(vars);
        terms.push_back(x);
        args.push_back({x.op == Expr::VAR, x.v});  // only meaningful for VAR / CONST
        if (peek(',')) {
          expect(",");
          continue;
        }
        break;
      }
    }
    expect(")");
    return {relation(name, (int)args.size()), args};
  }
  // A body item is an atom `name(...)` or a comparison `expr op expr`.
  bool next_is_atom() {
    skip();
    size_t save = i;
    bool atom = false;
    if (i < s.size() && (std::isalpha((unsigned char)s[i]) || s[i] == '_')) {
      (void)ident();
      atom = peek('(');
    }
    i = save;
    return atom;
  }
  Atom atom(std::map<std::string, int>& vars) {
    std::string name = ident();
    expect("(");
    std::vector<Term> args;
    if (!peek(')')) {
      for (;;) {
        skip();
        if (i < s.size() && std::isdigit((unsigned char)s[i])) {
          args.push_back({false, number()});
        } else {
          std::string v = ident();
          auto it = vars.find(v);
          int id = it == vars.end() ? (int)vars.size() : it->second;
          if (it == vars.end()) vars[v] = id;
          args.push_back({true, (uint32_t)id});
        }
        if (peek(',')) {
          expect(",");
          continue;
        }
        break;
      }
    }
    expect(")");
    return {relation(name, (int)args.size()), args};
  }
  void parse() {
    for (;;) {
      skip();
      if (i >= s.size()) break;
      if (s[i] == '.') {
        ++i;
        std::string kw = ident();
        std::string name = ident();
        expect("/");
        int arity = (int)number();
        if (arity < 0 || arity > 4) fail("arity must be 0..4");
        int r = relation(name, arity);
        if (kw == "input") prog.rels[r].input = true;
        else if (kw != "output") fail("unknown directive ." + kw);
        continue;
      }
      std::map<std::string, int> vars;
      Rule rule;
      rule.head = head(vars, rule.head_terms);
      expect(":-");
      for (;;) {
        if (next_is_atom()) rule.body.push_back(atom(vars));
        else rule.conds.push_back(comparison(vars));
        if (peek(',')) {
          expect(",");
          continue;
        }
        break;
      }
      expect(".");
      rule.nvars = (int)vars.size();
      std::vector<bool> inbody(rule.nvars, false);
      for (auto& a : rule.body)
        for (auto& t : a.args)
          if (t.var) inbody[t.v] = true;
      if (rule.body.empty()) fail("a rule needs a body atom");
      std::function<void(const Expr&)> bound = [&](const Expr& x) {
        if (x.op == Expr::VAR && !inbody[x.v]) fail("variable not bound by a body atom");
        for (auto& k : x.kids) bound(k);
      };
      for (auto& t : rule.head_terms) bound(t);
      for (auto& c : rule.conds) bound(c.a), bound(c.b);
      prog.rules.push_back(rule);
    }
    for (auto& r : prog.rules) prog.rels[r.head.rel].idb = true;
    for (auto& rel : prog.rels)
      if (rel.idb && rel.input) throw std::runtime_error("input relation " + rel.name + " has a rule");
    stratify();
  }
  // Strata: strongly connected components of the predicate dependency graph
  // over derived relations, in topological order; independent components in
  // order of first mention.
  void stratify() {
    int n = (int)prog.rels.size();
    std::vector<std::vector<char>> reach(n, std::vector<char>(n, 0));
    for (auto& r : prog.rules)
      for (auto& b : r.body) reach[b.rel][r.head.rel] = 1;
    for (int k = 0; k < n; ++k)
      for (int a = 0; a < n; ++a)
        if (reach[a][k])
          for (int b = 0; b < n; ++b)
            if (reach[k][b]) reach[a][b] = 1;
    std::vector<int> comp(n, -1);
    std::vector<std::vector<int>> comps;
    for (int a = 0; a < n; ++a) {
      if (!prog.rels[a].idb || comp[a] >= 0) continue;
      comp[a] = (int)comps.size();
      comps.push_back({a});
      for (int b = a + 1; b < n; ++b)
        if (prog.rels[b].idb && comp[b] < 0 && reach[a][b] && reach[b][a]) {
          comp[b] = comp[a];
          comps.back().push_back(b);
        }
    }
    std::vector<char> done(comps.size(), 0);
    for (size_t step = 0; step < comps.size(); ++step) {
      int pick = -1;
      for (size_t c = 0; c < comps.size(); ++c) {
        if (done[c]) continue;
        bool ready = true;
        for (size_t d = 0; d < comps.size() && ready; ++d) {
          if (d == c || done[d]) continue;
          if (reach[comps[d][0]][comps[c][0]]) ready = false;
        }
        if (ready && (pick < 0 || prog.rels[comps[c][0]].first_seen < prog.rels[comps[pick][0]].first_seen))
          pick = (int)c;
      }
      done[pick] = 1;
      std::vector<int> rules;
      for (size_t ri = 0; ri < prog.rules.size(); ++ri)
        if (comp[prog.rules[ri].head.rel] == pick) rules.push_back((int)ri);
      prog.strata.push_back(rules);
    }
  }
};

// ----------------------------------------------------------------- semiring
const int KMAX = 3;
const int WMAX = 4;  // words of a proof's fact set: up to 256 probabilistic facts per sample
// A proof: the set of its facts, fact f at bit f % 64 of word f / 64.  Sets
// are ordered as the unsigned integers they spell (highest word first).
struct Bits {
  uint64_t w[WMAX] = {0, 0, 0, 0};
  bool test(int f) const { return (w[f >> 6] >> (f & 63)) & 1ull; }
  void set(int f) { w[f >> 6] |= 1ull << (f & 63); }
  Bits operator|(const Bits& o) const {
    Bits r;
    for (int i = 0; i < WMAX; ++i) r.w[i] = w[i] | o.w[i];
    return r;
  }
  bool operator==(const Bits& o) const {
    for (int i = 0; i < WMAX; ++i)
      if (w[i] != o.w[i]) return false;
    return true;
  }
  bool operator!=(const Bits& o) const { return !(*this == o); }
  bool operator<(const Bits& o) const {
    for (int i = WMAX - 1; i >= 0; --i)
      if (w[i] != o.w[i]) return w[i] < o.w[i];
    return false;
  }
};
struct Tag {
  double v = 0;
  uint32_t fid = 0;  // differentiable max-min: the input fact the value comes from
  int cnt = 0;
  Bits bits[KMAX];
  float p[KMAX] = {0, 0, 0};
};

struct Semiring {
  int kind;
  int k;
  bool converge() const { return kind != REF_ADDMULT && kind != REF_DIFF_ADDMULT; }
  bool topk() const { return kind == REF_TOPK || kind == REF_DIFF_TOPK; }

  // Probability of a proof (conjunction of the facts whose bits are set):
  // product of their probabilities in binary32, facts in ascending id order,
  // starting from 1.
  static float proof_prob(const Bits& b, const std::vector<float>& q) {
    float acc = 1.0f;
    for (int i = 0; i < 64 * WMAX; ++i)
      if (b.test(i)) acc = acc * q[i];
    return acc;
  }
  // Keep the k best distinct proofs: probability descending, then the bitset
  // as an unsigned integer ascending.
  Tag best(std::vector<Bits> cand, const std::vector<float>& q) const {
    std::sort(cand.begin(), cand.end());
    cand.erase(std::unique(cand.begin(), cand.end()), cand.end());
    std::vector<std::pair<float, Bits>> ranked;
    for (const Bits& b : cand) ranked.push_back({proof_prob(b, q), b});
    std::sort(ranked.begin(), ranked.end(), [](const std::pair<float, Bits>& a, const std::pair<float, Bits>& b) {
      if (a.first != b.first) return a.first > b.first;
      return a.second < b.second;
    });
    Tag t;
    t.cnt = (int)std::min<size_t>(ranked.size(), (size_t)k);
    for (int i = 0; i < t.cnt; ++i) {
      t.bits[i] = ranked[i].second;
      t.p[i] = ranked[i].first;
    }
    return t;
  }
  Tag zero() const {
    Tag t;
    if (kind == REF_MINPLUS) t.v = std::numeric_limits<double>::infinity();
    return t;
  }
  // differentiable max-min: the smaller (times) or larger (plus) value; on
  // equal values the smaller fact number
  static Tag pick(const Tag& a, const Tag& b, bool larger) {
    if (a.v != b.v) return (a.v > b.v) == larger ? a : b;
    return a.fid <= b.fid ? a : b;
  }
  Tag otimes(const Tag& a, const Tag& b, const std::vector<float>& q) const {
    Tag t;
    switch (kind) {
      case REF_BOOL: t.v = 1; break;
      case REF_MAXMIN: t.v = std::min(a.v, b.v); break;
      case REF_MINPLUS: t.v = a.v + b.v; break;
      case REF_ADDMULT:
      case REF_DIFF_ADDMULT: t.v = a.v * b.v; break;
      case REF_DIFF_MAXMIN: t = pick(a, b, false); break;
      default: {
        std::vector<Bits> cand;
        for (int i = 0; i < a.cnt; ++i)
          for (int j = 0; j < b.cnt; ++j) cand.push_back(a.bits[i] | b.bits[j]);
        t = best(cand, q);
      }
    }
    return t;
  }
  Tag oplus(const Tag& a, const Tag& b, const std::vector<float>& q) const {
    Tag t;
    switch (kind) {
      case REF_BOOL: t.v = 1; break;
      case REF_MAXMIN: t.v = std::max(a.v, b.v); break;
      case REF_MINPLUS: t.v = std::min(a.v, b.v); break;
      case REF_ADDMULT:
      case REF_DIFF_ADDMULT: t.v = std::min(1.0, a.v + b.v); break;
      case REF_DIFF_MAXMIN: t = pick(a, b, true); break;
      default: {
        std::vector<Bits> cand;
        for (int i = 0; i < a.cnt; ++i) cand.push_back(a.bits[i]);
        for (int j = 0; j < b.cnt; ++j) cand.push_back(b.bits[j]);
        t = best(cand, q);
      }
    }
    return t;
  }
  bool same(const Tag& a, const Tag& b) const {
    if (kind == REF_BOOL) return true;
    if (kind == REF_DIFF_MAXMIN) return a.v == b.v && a.fid == b.fid;
    if (!topk()) return a.v == b.v;
    if (a.cnt != b.cnt) return false;
    for (int i = 0; i < a.cnt; ++i)
      if (a.bits[i] != b.bits[i]) return false;
    return true;
  }
};

// Exact probability of the disjunction of the kept proofs, facts independent:
// inclusion-exclusion over the non-empty subsets of proofs.
double incl_excl(const Tag& t, const std::vector<float>& q) {
  double P = 0;
  for (int S = 1; S < (1 << t.cnt); ++S) {
    Bits u;
    int sz = 0;
    for (int i = 0; i < t.cnt; ++i)
      if (S >> i & 1) {
        u = u | t.bits[i];
        ++sz;
      }
    double prod = 1;
    for (int b = 0; b < 64 * WMAX; ++b)
      if (u.test(b)) prod *= (double)q[b];
    P += (sz % 2 ? 1.0 : -1.0) * prod;
  }
  return P;
}

// ----------------------------------------------------------------- database
using Key = std::vector<uint32_t>;
struct Entry {
  Tag tag;
  int stratum = -1;  // -1: input fact
  int round = 0;
  double s = 0;  // add-mult: unclamped sum of the discovery derivations
  double adj = 0;
  std::vector<std::vector<Entry*>> derivs;  // diff add-mult discovery derivations
  std::vector<long> facts;                  // input facts merged into this entry
};
using Rel = std::map<Key, Entry>;

struct SampleDB {
  std::vector<Rel> rel;
  std::vector<float> q;                           // top-k fact probabilities by local id
  std::vector<std::pair<int, long>> fact_of_bit;  // local id -> (relation, fact index)
  std::vector<int> rounds;                        // per stratum
};

struct Cand {
  Tag tag;
  bool any = false;
  double s = 0;
  std::vector<std::vector<Entry*>> derivs;
};

}  // namespace

struct ref_engine {
  Program prog;
  Semiring sr;
  bool batched = false;
  bool ran = false;
  std::map<uint32_t, SampleDB> samples;
  std::vector<long> nfacts;                       // per relation
  std::vector<std::vector<double>> grad;          // per relation, per fact
  std::vector<std::vector<uint32_t>> fact_sample; // per relation, per fact
  std::vector<std::pair<int, long>> fact_of_fid;  // differentiable max-min: fact number -> (relation, fact)
  std::string err;
};

namespace {

struct Evaluator {
  ref_engine* e;
  SampleDB& db;
  int stratum;
  int round;
  // per round lookup tables: (rel, bound mask) -> bound values -> entries
  std::map<std::pair<int, unsigned>, std::map<Key, std::vector<std::pair<const Key*, Entry*>>>> index;
  std::vector<std::map<Key, Cand>> cand;

  const std::map<Key, std::vector<std::pair<const Key*, Entry*>>>& lookup(int rel, unsigned mask) {
    auto k = std::make_pair(rel, mask);
    auto it = index.find(k);
    if (it != index.end()) return it->second;
    auto& m = index[k];
    int ar = e->prog.rels[rel].arity;
    for (auto& kv : db.rel[rel]) {
      Key b;
      for (int p = 0; p < ar; ++p)
        if (mask >> p & 1u) b.push_back(kv.first[p]);
      m[b].push_back({&kv.first, &kv.second});
    }
    return m;
  }

  static uint32_t eval(const Expr& x, const std::vector<uint32_t>& val, bool& ok) {
    switch (x.op) {
      case Expr::VAR: return val[x.v];
      case Expr::CONST: return x.v;
      default: break;
    }
    const uint32_t a = eval(x.kids[0], val, ok), b = eval(x.kids[1], val, ok);
    switch (x.op) {
      case Expr::ADD: return a + b;
      case Expr::SUB: return a - b;
      case Expr::MUL: return a * b;
      default:
        if (b == 0) {
          ok = false;
          return 0;
        }
        return x.op == Expr::DIV ? a / b : a % b;
    }
  }
  static bool holds(const Cond& c, const std::vector<uint32_t>& val) {
    bool ok = true;
    const uint32_t a = eval(c.a, val, ok), b = eval(c.b, val, ok);
    if (!ok) return false;
    switch (c.cmp) {
      case CMP_EQ: return a == b;
      case CMP_NE: return a != b;
      case CMP_LT: return a < b;
      case CMP_LE: return a <= b;
      case CMP_GT: return a > b;
      default: return a >= b;
    }
  }

  void produce(const Rule& r, const std::vector<uint32_t>& val, const std::vector<Entry*>& body) {
    for (const Cond& c : r.conds)
      if (!holds(c, val)) return;
    Key h;
    bool ok = true;
    for (auto& t : r.head_terms) h.push_back(eval(t, val, ok));
    if (!ok) return;
    Rel& target = db.rel[r.head.rel];
    bool present = target.count(h) != 0;
    const Semiring& sr = e->sr;
    if (!sr.converge() && present) return;  // frozen: later derivations ignored
    Tag v = body[0]->tag;
    for (size_t j = 1; j < body.size(); ++j) v = sr.otimes(v, body[j]->tag, db.q);
    Cand& c = cand[r.head.rel][h];
    if (sr.converge()) {
      c.tag = c.any ? sr.oplus(c.tag, v, db.q) : v;
    } else {
      c.s += v.v;
      if (sr.kind == REF_DIFF_ADDMULT) c.derivs.push_back(body);
    }
    c.any = true;
  }

  void enumerate(const Rule& r, size_t j, std::vector<uint32_t>& val, std::vector<char>& bound,
                 std::vector<Entry*>& body) {
    if (j == r.body.size()) {
      produce(r, val, body);
      return;
    }
    const Atom& a = r.body[j];
    unsigned mask = 0;
    Key want;
    for (size_t p = 0; p < a.args.size(); ++p) {
      const Term& t = a.args[p];
      if (!t.var) {
        mask |= 1u << p;
        want.push_back(t.v);
      } else if (bound[t.v]) {
        mask |= 1u << p;
        want.push_back(val[t.v]);
      }
    }
    auto visit = [&](const Key& key, Entry* ent) {
      std::vector<uint32_t> v2 = val;
      std::vector<char> b2 = bound;
      for (size_t p = 0; p < a.args.size(); ++p) {
        const Term& t = a.args[p];
        if (!t.var) {
          if (key[p] != t.v) return;
        } else if (b2[t.v]) {
          if (key[p] != v2[t.v]) return;
        } else {
          v2[t.v] = key[p];
          b2[t.v] = 1;
        }
      }
      body.push_back(ent);
      enumerate(r, j + 1, v2, b2, body);
      body.pop_back();
    };
    if (mask == 0) {
      for (auto& kv : db.rel[a.rel]) visit(kv.first, &kv.second);
    } else {
      const auto& m = lookup(a.rel, mask);
      auto it = m.find(want);
      if (it == m.end()) return;
      for (auto& pr : it->second) visit(*pr.first, pr.second);
    }
  }

  // One naive Jacobi round; returns whether anything changed.
  bool step(const std::vector<int>& rules) {
    index.clear();
    cand.assign(e->prog.rels.size(), {});
    for (int ri : rules) {
      const Rule& r = e->prog.rules[ri];
      std::vector<uint32_t> val(r.nvars, 0);
      std::vector<char> bound(r.nvars, 0);
      std::vector<Entry*> body;
      enumerate(r, 0, val, bound, body);
    }
    index.clear();
    const Semiring& sr = e->sr;
    bool changed = false;
    for (size_t rel = 0; rel < cand.size(); ++rel) {
      for (auto& kv : cand[rel]) {
        Rel& target = db.rel[rel];
        auto it = target.find(kv.first);
        if (sr.converge()) {
          if (it == target.end()) {
            Entry en;
            en.tag = kv.second.tag;
            en.stratum = stratum;
            en.round = round;
            target.emplace(kv.first, en);
            changed = true;
          } else {
            Tag t2 = sr.oplus(it->second.tag, kv.second.tag, db.q);
            if (!sr.same(t2, it->second.tag)) {
              it->second.tag = t2;
              changed = true;
            }
          }
        } else if (it == target.end()) {
          Entry en;
          en.s = kv.second.s;
          en.tag.v = std::min(1.0, kv.second.s);
          en.stratum = stratum;
          en.round = round;
          en.derivs = std::move(kv.second.derivs);
          target.emplace(kv.first, std::move(en));
          changed = true;
        }
      }
    }
    return changed;
  }
};

void run_sample(ref_engine* e, SampleDB& db) {
  db.rounds.assign(e->prog.strata.size(), 0);
  for (size_t st = 0; st < e->prog.strata.size(); ++st) {
    Evaluator ev{e, db, (int)st, 0, {}, {}};
    for (int round = 1;; ++round) {
      ev.round = round;
      if (!ev.step(e->prog.strata[st])) {
        db.rounds[st] = round;
        break;
      }
    }
  }
}

}  // namespace

extern "C" {

int ref_create(const char* program, int semiring, int k, int batched, ref_engine** out, char* err,
               size_t errlen) {
  *out = nullptr;
  if (semiring < REF_BOOL || semiring > REF_DIFF_MAXMIN || k < 1 || k > KMAX) {
    if (err && errlen) std::snprintf(err, errlen, "bad semiring or k");
    return 1;
  }
  try {
    Parser p;
    p.s = program;
    p.parse();
    auto* e = new ref_engine();
    e->prog = std::move(p.prog);
    e->sr = Semiring{semiring, k};
    e->batched = batched != 0;
    e->nfacts.assign(e->prog.rels.size(), 0);
    e->grad.assign(e->prog.rels.size(), {});
    e->fact_sample.assign(e->prog.rels.size(), {});
    *out = e;
    return 0;
  } catch (const std::exception& ex) {
    if (err && errlen) std::snprintf(err, errlen, "%s", ex.what());
    return 1;
  }
}

static SampleDB& sample_db(ref_engine* e, uint32_t s) {
  auto it = e->samples.find(s);
  if (it != e->samples.end()) return it->second;
  SampleDB& db = e->samples[s];
  db.rel.assign(e->prog.rels.size(), {});
  return db;
}

int ref_add_facts(ref_engine* e, const char* rel, size_t n, const uint32_t* sample_ids,
                  const uint32_t* cols, const float* tags) {
  int r = e->prog.find(rel);
  if (r < 0 || !e->prog.rels[r].input) {
    e->err = std::string("not an input relation: ") + rel;
    return 1;
  }
  if (e->ran) {
    e->err = "facts added after run";
    return 1;
  }
  if (e->sr.kind != REF_BOOL && !tags) {
    e->err = "tags required";
    return 1;
  }
  int ar = e->prog.rels[r].arity;
  for (size_t i = 0; i < n; ++i) {
    uint32_t s = (e->batched && sample_ids) ? sample_ids[i] : 0;
    SampleDB& db = sample_db(e, s);
    long f = e->nfacts[r]++;
    e->fact_sample[r].push_back(s);
    Key key(cols + i * ar, cols + (i + 1) * ar);
    Tag t;
    if (e->sr.topk()) {
      if (db.q.size() >= 64 * WMAX) {
        e->err = "more than 256 probabilistic facts in one sample";
        return 2;
      }
      t.cnt = 1;
      t.bits[0].set((int)db.q.size());
      t.p[0] = tags[i];
      db.q.push_back(tags[i]);
      db.fact_of_bit.push_back({r, f});
    } else if (e->sr.kind == REF_DIFF_MAXMIN) {
      t.v = (double)tags[i];
      t.fid = (uint32_t)e->fact_of_fid.size();
      e->fact_of_fid.push_back({r, f});
    } else if (e->sr.kind != REF_BOOL) {
      t.v = (double)tags[i];
    } else {
      t.v = 1;
    }
    auto it = db.rel[r].find(key);
    if (it == db.rel[r].end()) {
      Entry en;
      en.tag = t;
      en.s = t.v;
      en.facts.push_back(f);
      db.rel[r].emplace(key, en);
    } else {
      it->second.facts.push_back(f);
      it->second.s += t.v;
      it->second.tag = e->sr.oplus(it->second.tag, t, db.q);
    }
  }
  return 0;
}

int ref_run(ref_engine* e) {
  for (auto& kv : e->samples) run_sample(e, kv.second);
  if (e->samples.empty()) {
    // no facts at all: still define round counts
    SampleDB& db = sample_db(e, 0);
    run_sample(e, db);
  }
  e->ran = true;
  for (size_t r = 0; r < e->prog.rels.size(); ++r) e->grad[r].assign(e->nfacts[r], 0.0);
  return 0;
}

long ref_size(ref_engine* e, const char* rel) {
  int r = e->prog.find(rel);
  if (r < 0) return -1;
  long n = 0;
  for (auto& kv : e->samples) n += (long)kv.second.rel[r].size();
  return n;
}

int ref_num_strata(ref_engine* e) { return (int)e->prog.strata.size(); }

int ref_rounds(ref_engine* e, int stratum) {
  if (stratum < 0 || stratum >= (int)e->prog.strata.size()) return -1;
  int m = 0;
  for (auto& kv : e->samples) m = std::max(m, kv.second.rounds[stratum]);
  return m;
}

int ref_read(ref_engine* e, const char* rel, uint32_t* sample_ids, uint32_t* cols, double* value,
             int32_t* cnt, uint64_t* bits, float* p, double* prob, int32_t* round_found) {
  int r = e->prog.find(rel);
  if (r < 0) return 1;
  int ar = e->prog.rels[r].arity;
  size_t i = 0;
  for (auto& kv : e->samples) {
    for (auto& t : kv.second.rel[r]) {
      if (sample_ids) sample_ids[i] = kv.first;
      if (cols)
        for (int c = 0; c < ar; ++c) cols[i * ar + c] = t.first[c];
      if (value) value[i] = e->sr.kind == REF_BOOL ? 1.0 : t.second.tag.v;
      if (cnt) cnt[i] = t.second.tag.cnt;
      for (int j = 0; j < KMAX; ++j) {
        if (bits) bits[i * KMAX + j] = j < t.second.tag.cnt ? t.second.tag.bits[j].w[0] : 0;
        if (p) p[i * KMAX + j] = j < t.second.tag.cnt ? t.second.tag.p[j] : 0.0f;
      }
      if (prob) prob[i] = e->sr.topk() ? incl_excl(t.second.tag, kv.second.q) : t.second.tag.v;
      if (round_found) round_found[i] = t.second.round;
      ++i;
    }
  }
  return 0;
}

int ref_read_bits(ref_engine* e, const char* rel, uint64_t* bits) {
  int r = e->prog.find(rel);
  if (r < 0) return 1;
  size_t i = 0;
  for (auto& kv : e->samples)
    for (auto& t : kv.second.rel[r]) {
      for (int j = 0; j < KMAX; ++j)
        for (int w = 0; w < WMAX; ++w)
          bits[(i * KMAX + j) * WMAX + w] = j < t.second.tag.cnt ? t.second.tag.bits[j].w[w] : 0;
      ++i;
    }
  return 0;
}

void ref_zero_grad(ref_engine* e) {
  for (auto& g : e->grad) std::fill(g.begin(), g.end(), 0.0);
}

int ref_backward(ref_engine* e, const char* out_rel, const double* grad_out) {
  int r = e->prog.find(out_rel);
  if (r < 0 || !e->ran) return 1;
  int kind = e->sr.kind;
  if (kind != REF_DIFF_ADDMULT && kind != REF_DIFF_TOPK && kind != REF_DIFF_MAXMIN) {
    e->err = "backward needs a differentiable semiring";
    return 1;
  }
  size_t i = 0;
  for (auto& kv : e->samples) {
    SampleDB& db = kv.second;
    if (kind == REF_DIFF_MAXMIN) {
      // the tag is the probability of one input fact: derivative 1 there
      for (auto& t : db.rel[r]) {
        const auto fr = e->fact_of_fid[t.second.tag.fid];
        e->grad[fr.first][fr.second] += grad_out[i++];
      }
      continue;
    }
    if (kind == REF_DIFF_TOPK) {
      // dP/dq_j of the inclusion-exclusion probability, proofs held fixed.
      for (auto& t : db.rel[r]) {
        double g = grad_out[i++];
        const Tag& tg = t.second.tag;
        for (int S = 1; S < (1 << tg.cnt); ++S) {
          Bits u;
          int sz = 0;
          for (int a = 0; a < tg.cnt; ++a)
            if (S >> a & 1) {
              u = u | tg.bits[a];
              ++sz;
            }
          double sign = sz % 2 ? 1.0 : -1.0;
          for (int j = 0; j < 64 * WMAX; ++j) {
            if (!u.test(j)) continue;
            double prod = 1;
            for (int b = 0; b < 64 * WMAX; ++b)
              if (b != j && u.test(b)) prod *= (double)db.q[b];
            auto fr = db.fact_of_bit[j];
            e->grad[fr.first][fr.second] += g * sign * prod;
          }
        }
      }
      continue;
    }
    // diff add-mult: reverse sweep over the discovery derivations.
    for (auto& rel : db.rel)
      for (auto& t : rel) t.second.adj = 0;
    for (auto& t : db.rel[r]) t.second.adj += grad_out[i++];
    std::vector<Entry*> order;
    for (auto& rel : db.rel)
      for (auto& t : rel)
        if (t.second.stratum >= 0) order.push_back(&t.second);
    std::stable_sort(order.begin(), order.end(), [](const Entry* a, const Entry* b) {
      if (a->stratum != b->stratum) return a->stratum > b->stratum;
      return a->round > b->round;
    });
    for (Entry* t : order) {
      if (!(t->s < 1.0)) continue;  // clamp: zero derivative once the sum reaches 1
      double g = t->adj;
      for (auto& d : t->derivs) {
        for (size_t j = 0; j < d.size(); ++j) {
          double prod = 1;
          for (size_t k = 0; k < d.size(); ++k)
            if (k != j) prod *= d[k]->tag.v;
          d[j]->adj += g * prod;
        }
      }
    }
    for (size_t rr = 0; rr < db.rel.size(); ++rr) {
      if (!e->prog.rels[rr].input) continue;
      for (auto& t : db.rel[rr]) {
        double g = t.second.s < 1.0 ? t.second.adj : 0.0;
        for (long f : t.second.facts) e->grad[rr][f] += g;
      }
    }
  }
  return 0;
}

int ref_read_fid(ref_engine* e, const char* rel, uint32_t* fid) {
  int r = e->prog.find(rel);
  if (r < 0) return 1;
  size_t i = 0;
  for (auto& kv : e->samples)
    for (auto& t : kv.second.rel[r]) fid[i++] = t.second.tag.fid;
  return 0;
}

int ref_vid_op(int op, double av, uint32_t aid, double bv, uint32_t bid, double* ov, uint32_t* oid) {
  Tag a, b;
  a.v = av;
  a.fid = aid;
  b.v = bv;
  b.fid = bid;
  const Tag t = Semiring::pick(a, b, op == 0);
  *ov = t.v;
  *oid = t.fid;
  return 0;
}

int ref_read_grad(ref_engine* e, const char* in_rel, double* grad_in) {
  int r = e->prog.find(in_rel);
  if (r < 0 || !e->ran) return 1;
  std::copy(e->grad[r].begin(), e->grad[r].end(), grad_in);
  return 0;
}

const char* ref_error(ref_engine* e) { return e->err.c_str(); }

void ref_free(ref_engine* e) { delete e; }

int ref_scalar_op(int semiring, int op, double a, double b, double* out) {
  if (semiring < REF_BOOL || semiring > REF_DIFF_ADDMULT) return 1;
  Semiring sr{semiring, 1};
  Tag x, y;
  x.v = a;
  y.v = b;
  std::vector<float> q;
  *out = (op ? sr.otimes(x, y, q) : sr.oplus(x, y, q)).v;
  return 0;
}

int ref_scalar_identity(int semiring, int which, double* out) {
  if (semiring < REF_BOOL || semiring > REF_DIFF_ADDMULT) return 1;
  Semiring sr{semiring, 1};
  if (which == 0) *out = sr.zero().v;  // absorbing for x, neutral for +
  else *out = semiring == REF_MINPLUS ? 0.0 : 1.0;
  return 0;
}

int ref_topk_op(int k, int op, int acnt, const uint64_t* abits, int bcnt, const uint64_t* bbits, const float* q,
                int* ocnt, uint64_t* obits, float* oprob) {
  if (k < 1 || k > KMAX || acnt < 0 || acnt > KMAX || bcnt < 0 || bcnt > KMAX) return 1;
  Semiring sr{REF_TOPK, k};
  std::vector<float> qv(q, q + 64);
  Tag a, b;
  a.cnt = acnt;
  b.cnt = bcnt;
  for (int i = 0; i < acnt; ++i) {
    a.bits[i].w[0] = abits[i];
    a.p[i] = Semiring::proof_prob(a.bits[i], qv);
  }
  for (int i = 0; i < bcnt; ++i) {
    b.bits[i].w[0] = bbits[i];
    b.p[i] = Semiring::proof_prob(b.bits[i], qv);
  }
  Tag t = op ? sr.otimes(a, b, qv) : sr.oplus(a, b, qv);
  *ocnt = t.cnt;
  for (int i = 0; i < KMAX; ++i) {
    obits[i] = i < t.cnt ? t.bits[i].w[0] : 0;
    oprob[i] = i < t.cnt ? t.p[i] : 0.0f;
  }
  return 0;
}

}  // extern "C"
