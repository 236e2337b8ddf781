// Parser, stratifier and join planner for the supported Datalog fragment.
#include "program.h"

#include <algorithm>
#include <cctype>
#include <cstring>
#include <functional>
#include <map>
#include <stdexcept>

namespace dlfix {

int Program::find(const std::string& name) const {
  for (size_t i = 0; i < rels.size(); ++i)
    if (rels[i].name == name) return (int)i;
  return -1;
}

namespace {

struct Failure {
  int code;
  std::string msg;
};

class Reader {
 public:
  explicit Reader(const char* t) : s_(t) {}

  void run(Program& p) {
    for (;;) {
      skip();
      if (pos_ >= s_.size()) break;
      if (s_[pos_] == '.') {
        ++pos_;
        directive(p);
      } else {
        rule(p);
      }
    }
  }

 private:
  std::string s_;
  size_t pos_ = 0;
  int mentions_ = 0;
  std::map<uint32_t, int> const_vars_;  // constants of the rule being read -> their variable

  [[noreturn]] void parse_error(const std::string& m) {
    throw Failure{2, "parse error at offset " + std::to_string(pos_) + ": " + m};
  }
  void skip() {
    while (pos_ < s_.size()) {
      char c = s_[pos_];
      if (std::isspace((unsigned char)c)) {
        ++pos_;
      } else if (c == '#' || (c == '/' && pos_ + 1 < s_.size() && s_[pos_ + 1] == '/')) {
        while (pos_ < s_.size() && s_[pos_] != '\n') ++pos_;
      } else {
        return;
      }
    }
  }
  bool at(char c) {
    skip();
    return pos_ < s_.size() && s_[pos_] == c;
  }
  void eat(const char* tok) {
    skip();
    size_t n = std::strlen(tok);
    if (s_.compare(pos_, n, tok) != 0) parse_error(std::string("expected '") + tok + "'");
    pos_ += n;
  }
  std::string name() {
    skip();
    size_t b = pos_;
    if (pos_ < s_.size() && (std::isalpha((unsigned char)s_[pos_]) || s_[pos_] == '_'))
      while (pos_ < s_.size() && (std::isalnum((unsigned char)s_[pos_]) || s_[pos_] == '_')) ++pos_;
    if (b == pos_) parse_error("expected a name");
    return s_.substr(b, pos_ - b);
  }
  int integer() {
    skip();
    size_t b = pos_;
    long v = 0;
    while (pos_ < s_.size() && std::isdigit((unsigned char)s_[pos_]) && v < 1000000) v = v * 10 + (s_[pos_++] - '0');
    if (b == pos_) parse_error("expected an integer");
    return (int)v;
  }
  uint32_t u32() {
    skip();
    size_t b = pos_;
    uint64_t v = 0;
    while (pos_ < s_.size() && std::isdigit((unsigned char)s_[pos_])) {
      v = v * 10 + (uint64_t)(s_[pos_++] - '0');
      if (v > 0xffffffffull) parse_error("constant above 2^32 - 1");
    }
    if (b == pos_) parse_error("expected a constant");
    return (uint32_t)v;
  }
  bool digit() {
    skip();
    return pos_ < s_.size() && std::isdigit((unsigned char)s_[pos_]);
  }
  static int var_id(std::map<std::string, int>& vars, const std::string& v) {
    auto it = vars.find(v);
    if (it != vars.end()) return it->second;
    const int id = (int)vars.size();
    vars[v] = id;
    return id;
  }
  // A variable no name can clash with (names start with a letter or '_').
  static int fresh(std::map<std::string, int>& vars) { return var_id(vars, "#" + std::to_string(vars.size())); }
  void constant(Program& p, std::vector<Ins>& code, uint32_t v) {
    code.push_back({EV_CONST, (int32_t)v});
    p.max_const = std::max(p.max_const, v);
  }
  // Postfix code of an expression: sum := product {(+|-) product},
  // product := operand {(*|/|%) operand}, operand := constant | variable | ( sum ).
  void operand(Program& p, std::map<std::string, int>& vars, std::vector<Ins>& code) {
    if (at('(')) {
      eat("(");
      sum(p, vars, code);
      eat(")");
    } else if (digit()) {
      constant(p, code, u32());
    } else {
      code.push_back({EV_VAR, var_id(vars, name())});
    }
  }
  void product(Program& p, std::map<std::string, int>& vars, std::vector<Ins>& code) {
    operand(p, vars, code);
    for (;;) {
      EvalOp op;
      if (at('*')) op = EV_MUL;
      else if (at('/')) op = EV_DIV;
      else if (at('%')) op = EV_MOD;
      else return;
      ++pos_;
      operand(p, vars, code);
      code.push_back({op, 0});
    }
  }
  void sum(Program& p, std::map<std::string, int>& vars, std::vector<Ins>& code) {
    product(p, vars, code);
    for (;;) {
      EvalOp op;
      if (at('+')) op = EV_ADD;
      else if (at('-')) op = EV_SUB;
      else return;
      ++pos_;
      product(p, vars, code);
      code.push_back({op, 0});
    }
  }
  // lhs op rhs, appended to the rule's filter (conjunction)
  void comparison(Program& p, std::map<std::string, int>& vars, std::vector<Ins>& filter) {
    std::vector<Ins> code;
    sum(p, vars, code);
    skip();
    static const struct {
      const char* t;
      EvalOp op;
    } ops[] = {{"==", EV_EQ}, {"!=", EV_NE}, {"<=", EV_LE}, {">=", EV_GE}, {"<", EV_LT}, {">", EV_GT}, {"=", EV_EQ}};
    EvalOp op = EV_AND;
    for (auto& o : ops)
      if (s_.compare(pos_, std::strlen(o.t), o.t) == 0) {
        pos_ += std::strlen(o.t);
        op = o.op;
        break;
      }
    if (op == EV_AND) parse_error("expected a comparison operator");
    sum(p, vars, code);
    code.push_back({op, 0});
    const bool first = filter.empty();
    filter.insert(filter.end(), code.begin(), code.end());
    if (!first) filter.push_back({EV_AND, 0});
  }
  bool next_is_atom() {
    skip();
    const size_t save = pos_;
    bool atom = false;
    if (pos_ < s_.size() && (std::isalpha((unsigned char)s_[pos_]) || s_[pos_] == '_')) {
      (void)name();
      atom = at('(');
    }
    pos_ = save;
    return atom;
  }
  int relation(Program& p, const std::string& n, int arity) {
    int r = p.find(n);
    if (r < 0) {
      Relation rel;
      rel.name = n;
      rel.arity = arity;
      rel.first_mention = mentions_++;
      p.rels.push_back(rel);
      return (int)p.rels.size() - 1;
    }
    if (p.rels[r].arity != arity) parse_error("relation " + n + " used with two arities");
    return r;
  }
  void directive(Program& p) {
    std::string kw = name();
    std::string n = name();
    eat("/");
    int arity = integer();
    if (arity < 0 || arity > 4) throw Failure{3, "arity of " + n + " must be 0..4"};
    int r = relation(p, n, arity);
    if (kw == "input") p.rels[r].input = true;
    else if (kw != "output") parse_error("unknown directive ." + kw);
  }
  // A body atom.  A constant, or a variable already used in the same atom,
  // becomes a fresh variable with an equality condition (a selection).
  Atom atom(Program& p, std::map<std::string, int>& vars, std::vector<Ins>& filter) {
    std::string n = name();
    eat("(");
    Atom a;
    while (!at(')')) {
      int id;
      if (digit()) {
        // one variable per distinct constant of the rule: atoms that share a
        // constant join on it
        const uint32_t k = u32();
        auto it = const_vars_.find(k);
        if (it != const_vars_.end() && !std::count(a.vars.begin(), a.vars.end(), it->second)) {
          id = it->second;
        } else {
          id = fresh(vars);
          if (it == const_vars_.end()) const_vars_[k] = id;
          std::vector<Ins> eq{{EV_VAR, id}};
          constant(p, eq, k);
          eq.push_back({EV_EQ, 0});
          const bool first = filter.empty();
          filter.insert(filter.end(), eq.begin(), eq.end());
          if (!first) filter.push_back({EV_AND, 0});
        }
      } else {
        id = var_id(vars, name());
        if (std::count(a.vars.begin(), a.vars.end(), id)) {
          const int again = fresh(vars);
          const bool first = filter.empty();
          filter.insert(filter.end(), {{EV_VAR, again}, {EV_VAR, id}, {EV_EQ, 0}});
          if (!first) filter.push_back({EV_AND, 0});
          id = again;
        }
      }
      a.vars.push_back(id);
      if (!at(',')) break;
      eat(",");
    }
    eat(")");
    if (a.vars.size() > 4) throw Failure{3, "arity above 4"};
    a.rel = relation(p, n, (int)a.vars.size());
    return a;
  }
  // The head: every argument is an expression over the body's variables.
  Atom head(Program& p, std::map<std::string, int>& vars, std::vector<std::vector<Ins>>& code) {
    std::string n = name();
    eat("(");
    Atom a;
    while (!at(')')) {
      std::vector<Ins> c;
      sum(p, vars, c);
      if (c.size() == 1 && c[0].op == EV_VAR) {
        a.vars.push_back(c[0].arg);
        c.clear();
      } else {
        a.vars.push_back(-1);
      }
      code.push_back(c);
      if (!at(',')) break;
      eat(",");
    }
    eat(")");
    if (a.vars.size() > 4) throw Failure{3, "arity above 4"};
    a.rel = relation(p, n, (int)a.vars.size());
    return a;
  }
  void rule(Program& p) {
    std::map<std::string, int> vars;
    const_vars_.clear();
    Rule r;
    r.head = head(p, vars, r.head_code);
    eat(":-");
    for (;;) {
      if (next_is_atom()) r.body.push_back(atom(p, vars, r.filter));
      else comparison(p, vars, r.filter);
      if (at(',')) {
        eat(",");
        continue;
      }
      break;
    }
    eat(".");
    r.nvars = (int)vars.size();
    if (r.body.empty()) throw Failure{3, "a rule needs a body atom"};
    if (r.body.size() > 3) throw Failure{3, "more than 3 body atoms"};
    for (auto& b : r.body) {
      std::vector<int> v = b.vars;
      std::sort(v.begin(), v.end());
      if (std::adjacent_find(v.begin(), v.end()) != v.end())
        throw Failure{3, "repeated variable inside a body atom"};
    }
    auto bound = [&](int v) {
      for (auto& b : r.body)
        if (std::count(b.vars.begin(), b.vars.end(), v)) return true;
      return false;
    };
    for (int hv : r.head.vars)
      if (hv >= 0 && !bound(hv)) throw Failure{3, "head variable not bound by the body"};
    for (auto& c : r.head_code)
      for (auto& ins : c)
        if (ins.op == EV_VAR && !bound(ins.arg)) throw Failure{3, "head expression variable not bound by the body"};
    for (auto& ins : r.filter)
      if (ins.op == EV_VAR && !bound(ins.arg)) throw Failure{3, "condition variable not bound by the body"};
    p.rules.push_back(r);
  }
};

// Strongly connected components of the dependency graph (body -> head) over
// derived relations, emitted in dependency order, ties by first mention.
void stratify(Program& p) {
  const int n = (int)p.rels.size();
  std::vector<std::vector<char>> dep(n, std::vector<char>(n, 0));  // dep[a][b]: b depends on a
  for (auto& r : p.rules)
    for (auto& b : r.body) dep[b.rel][r.head.rel] = 1;
  for (int k = 0; k < n; ++k)
    for (int a = 0; a < n; ++a)
      if (dep[a][k])
        for (int b = 0; b < n; ++b)
          if (dep[k][b]) dep[a][b] = 1;
  std::vector<int> comp(n, -1);
  std::vector<std::vector<int>> comps;
  std::vector<int> order(n);
  for (int i = 0; i < n; ++i) order[i] = i;
  std::sort(order.begin(), order.end(), [&](int a, int b) { return p.rels[a].first_mention < p.rels[b].first_mention; });
  for (int a : order) {
    if (!p.rels[a].derived || comp[a] >= 0) continue;
    comp[a] = (int)comps.size();
    comps.push_back({a});
    for (int b : order)
      if (b != a && p.rels[b].derived && comp[b] < 0 && dep[a][b] && dep[b][a]) {
        comp[b] = comp[a];
        comps.back().push_back(b);
      }
  }
  std::vector<char> placed(comps.size(), 0);
  for (size_t step = 0; step < comps.size(); ++step) {
    int pick = -1;
    for (size_t c = 0; c < comps.size() && pick < 0; ++c) {  // comps are in first-mention order
      if (placed[c]) continue;
      bool ready = true;
      for (size_t d = 0; d < comps.size(); ++d)
        if (d != c && !placed[d] && dep[comps[d][0]][comps[c][0]]) ready = false;
      if (ready) pick = (int)c;
    }
    placed[pick] = 1;
    Stratum st;
    st.rels = comps[pick];
    for (int r : st.rels) p.rels[r].stratum = (int)p.strata.size();
    p.strata.push_back(st);
  }
}

int add_index(Program& p, const IndexSpec& ix) {
  for (size_t i = 0; i < p.indexes.size(); ++i)
    if (p.indexes[i] == ix) return (int)i;
  p.indexes.push_back(ix);
  return (int)p.indexes.size() - 1;
}

// stable_before: under frozen tags, same-stratum atoms before the delta atom
// read the stable part (full minus recent), so that every derivation with at
// least one recent atom is enumerated exactly once, by its first recent atom.
Plan make_plan(Program& p, int rule_id, int driver, bool delta, int recent_atom = -1, bool stable_before = false) {
  const Rule& r = p.rules[rule_id];
  Plan pl;
  pl.rule = rule_id;
  pl.head_rel = r.head.rel;
  pl.driver_atom = driver;
  pl.driver_rel = r.body[driver].rel;
  pl.delta = delta;
  pl.driver_vars = r.body[driver].vars;
  pl.max_cols = (int)std::max(r.body[driver].vars.size(), r.head.vars.size());
  std::vector<int> cur = r.body[driver].vars;
  std::vector<int> remaining;
  for (int j = 0; j < (int)r.body.size(); ++j)
    if (j != driver) remaining.push_back(j);
  auto has = [](const std::vector<int>& v, int x) { return std::find(v.begin(), v.end(), x) != v.end(); };
  // variables the evaluation at the plan's output reads
  std::vector<int> eval_vars;
  for (auto& c : r.head_code)
    for (auto& ins : c)
      if (ins.op == EV_VAR) eval_vars.push_back(ins.arg);
  for (auto& ins : r.filter)
    if (ins.op == EV_VAR) eval_vars.push_back(ins.arg);
  pl.eval = r.eval();
  // EV_VAR -> EV_SRC through `src_of` (the variable's column in the plan's
  // last table: >= 0 current table, < 0 index key position)
  auto resolve = [&](const std::function<int(int)>& src_of) {
    auto tr = [&](std::vector<Ins> code) {
      for (auto& ins : code)
        if (ins.op == EV_VAR) ins = Ins{EV_SRC, src_of(ins.arg)};
      return code;
    };
    pl.filter = tr(r.filter);
    pl.code.clear();
    for (auto& c : r.head_code) pl.code.push_back(tr(c));
  };
  if (remaining.empty()) {
    auto col = [&](int v) { return (int)(std::find(cur.begin(), cur.end(), v) - cur.begin()); };
    for (int hv : r.head.vars) pl.project.push_back(hv >= 0 ? col(hv) : 0);
    if (pl.eval) resolve(col);
    return pl;
  }
  while (!remaining.empty()) {
    int pick = -1;
    for (size_t i = 0; i < remaining.size() && pick < 0; ++i)
      for (int v : r.body[remaining[i]].vars)
        if (has(cur, v)) {
          pick = (int)i;
          break;
        }
    if (pick < 0) throw Failure{3, "a body atom shares no variable with the atoms before it"};
    const Atom& a = r.body[remaining[pick]];
    Step st;
    st.body_pos = remaining[pick];
    remaining.erase(remaining.begin() + pick);
    IndexSpec ix;
    ix.rel = a.rel;
    ix.recent = st.body_pos == recent_atom;
    ix.stable = stable_before && st.body_pos < driver && p.rels[a.rel].derived &&
                p.rels[a.rel].stratum == p.rels[r.head.rel].stratum;
    for (size_t c = 0; c < a.vars.size(); ++c)
      if (has(cur, a.vars[c])) {
        ix.perm.push_back((int)c);
        st.join_src.push_back((int)(std::find(cur.begin(), cur.end(), a.vars[c]) - cur.begin()));
      }
    ix.w = (int)ix.perm.size();
    for (size_t c = 0; c < a.vars.size(); ++c)
      if (!has(cur, a.vars[c])) ix.perm.push_back((int)c);
    st.index = add_index(p, ix);
    // variables needed after this step
    std::vector<int> need = r.head.vars;
    need.insert(need.end(), eval_vars.begin(), eval_vars.end());
    for (int j : remaining)
      for (int v : r.body[j].vars) need.push_back(v);
    std::vector<int> out;
    if (remaining.empty()) {
      out = r.head.vars;  // -1: a computed column
    } else {
      for (int v : cur)
        if (has(need, v) && !has(out, v)) out.push_back(v);
      for (int v : a.vars)
        if (has(need, v) && !has(out, v)) out.push_back(v);
    }
    auto src_of = [&](int v) {
      if (has(cur, v)) return (int)(std::find(cur.begin(), cur.end(), v) - cur.begin());
      int col = (int)(std::find(a.vars.begin(), a.vars.end(), v) - a.vars.begin());
      int kpos = (int)(std::find(ix.perm.begin(), ix.perm.end(), col) - ix.perm.begin());
      return -1 - kpos;
    };
    for (int v : out) st.out_src.push_back(v >= 0 ? src_of(v) : 0);
    if (remaining.empty() && pl.eval) resolve(src_of);
    st.out_vars = out;
    pl.max_cols = std::max(pl.max_cols, (int)out.size());
    pl.steps.push_back(st);
    cur = out;
  }
  return pl;
}

void plan(Program& p, bool frozen, bool diff) {
  for (auto& r : p.rules) p.rels[r.head.rel].derived = true;
  for (auto& rel : p.rels)
    if (rel.derived && rel.input) throw Failure{3, "input relation " + rel.name + " is the head of a rule"};
  stratify(p);
  for (size_t ri = 0; ri < p.rules.size(); ++ri) {
    const Rule& r = p.rules[ri];
    int s = p.rels[r.head.rel].stratum;
    if (diff && r.body.size() > 2) throw Failure{3, "differentiable add-mult supports at most 2 body atoms"};
    std::vector<int> same;
    for (int j = 0; j < (int)r.body.size(); ++j)
      if (p.rels[r.body[j].rel].derived && p.rels[r.body[j].rel].stratum == s) same.push_back(j);
    if (same.empty()) {
      p.plans.push_back(make_plan(p, (int)ri, 0, false));
      p.strata[s].base_plans.push_back((int)p.plans.size() - 1);
    } else {
      p.strata[s].recursive = true;
      for (int j : same) {
        p.plans.push_back(make_plan(p, (int)ri, j, true, -1, frozen && same.size() > 1));
        const int id = (int)p.plans.size() - 1;
        p.strata[s].delta_plans.push_back(id);
        if (r.body.size() == 2 && same.size() == 1) {
          p.plans.push_back(make_plan(p, (int)ri, 1 - j, false, j));
          p.plans[id].alt = (int)p.plans.size() - 1;
        }
      }
    }
  }
  p.max_cols = 0;
  for (auto& rel : p.rels) p.max_cols = std::max(p.max_cols, rel.arity);
  for (auto& pl : p.plans) p.max_cols = std::max(p.max_cols, pl.max_cols);
}

}  // namespace

int parse_and_plan(const char* text, bool frozen_tags, bool diff_lineage, Program& out, std::string& err) {
  try {
    Program p;
    Reader(text).run(p);
    if (p.rules.empty()) throw Failure{2, "program has no rules"};
    plan(p, frozen_tags, diff_lineage);
    out = std::move(p);
    return 0;
  } catch (const Failure& f) {
    err = f.msg;
    return f.code;
  }
}

}  // namespace dlfix
