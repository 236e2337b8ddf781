// Program text -> rules -> strata -> fixed-function join plans (host only).
//
// A plan evaluates one rule with one chosen "driver" atom: the driver's rows
// are expanded by a chain of binary index joins, one per remaining body atom
// (join lowering of Sec. 3.3 / Appendix A: build an index on one side, count
// matches per probe row, scan the counts, emit index pairs and gather
// columns and x-multiplied tags).  Base plans run once, in the first round of
// a stratum, with the first body atom as driver; delta plans run in later
// rounds with an atom of the rule's own stratum as driver, reading only that
// relation's recent tuples (semi-naive evaluation, Sec. 3.4).
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace dlfix {

struct Atom {
  int rel;
  std::vector<int> vars;  // variable per column (head: -1 where the column is computed)
};

// Expression evaluation (Sec. 5, bytecode interpreter; Sec. 3.3 eval<alpha>
// in the lowering of Project): a postfix program for a small stack machine
// over u32 values.  Operands are the rule's variables (VAR, arg = variable
// id; after planning: SRC, arg = column of the current table if >= 0, of the
// index row if < 0 as -1 - key position) and constants.  + - * wrap modulo
// 2^32, / and % are unsigned and void the derivation when the divisor is 0,
// comparisons are unsigned and push 0 or 1.
enum EvalOp : uint8_t {
  EV_VAR = 0, EV_SRC, EV_CONST, EV_ADD, EV_SUB, EV_MUL, EV_DIV, EV_MOD,
  EV_EQ, EV_NE, EV_LT, EV_LE, EV_GT, EV_GE, EV_AND
};
struct Ins {
  EvalOp op;
  int32_t arg = 0;  // variable / source (VAR, SRC) or constant (CONST, as u32)
};

struct Rule {
  Atom head;
  std::vector<std::vector<Ins>> head_code;  // per head column: empty = the plain variable head.vars[c]
  std::vector<Ins> filter;                  // empty = no condition; else pushes 1 when the derivation counts
  std::vector<Atom> body;
  int nvars = 0;
  bool eval() const {
    if (!filter.empty()) return true;
    for (auto& c : head_code)
      if (!c.empty()) return true;
    return false;
  }
};

struct Relation {
  std::string name;
  int arity = 0;
  bool input = false;
  bool derived = false;
  int stratum = -1;      // derived relations only
  int first_mention = 0;
};

// Index on a relation: its rows re-packed with the columns in `perm` order;
// the first `w` of them are the join columns, and a CSR offset array over the
// (sample, join columns) prefix gives every probe its range of matches.
struct IndexSpec {
  int rel;
  std::vector<int> perm;
  int w;
  bool recent = false;  // index over the relation's recent tuples (rebuilt every round)
  bool stable = false;  // index over full minus recent (the relation before the last round)
  bool identity() const {
    for (size_t i = 0; i < perm.size(); ++i)
      if (perm[i] != (int)i) return false;
    return true;
  }
  bool operator==(const IndexSpec& o) const {
    return rel == o.rel && perm == o.perm && w == o.w && recent == o.recent && stable == o.stable;
  }
};

// One binary join: current table (layout `in_vars`) x index rows.
struct Step {
  int index;                    // into Plan-set index list
  std::vector<int> join_src;    // per join column (index key order): column of the current table
  std::vector<int> out_src;     // per output column: >= 0 current-table column, < 0: index column (-1 - c)
  std::vector<int> out_vars;    // variables of the output layout (head columns for the last step)
  int body_pos;                 // body position of the joined atom
};

struct Plan {
  int rule;
  int head_rel;
  int driver_atom;              // body position of the driver
  int driver_rel;
  bool delta;                   // driver reads recent tuples (false: the whole relation)
  std::vector<int> driver_vars;
  std::vector<Step> steps;
  std::vector<int> project;     // no steps: head column j <- driver column project[j]
  int max_cols;                 // widest table of the plan
  // Evaluation at the plan's output (the last step, or the projection when
  // there are no steps): `filter` and the computed head columns, with EV_SRC
  // operands; head column c is computed when code[c] is non-empty.
  bool eval = false;
  std::vector<Ins> filter;
  std::vector<std::vector<Ins>> code;
  // Delta plans of 2-atom rules whose other atom is static also get a
  // "static-driven" twin: the static relation drives and the recent tuples
  // are the indexed side (same derivations, output grouped by the static
  // side's columns).  alt = plan id of the twin, -1 if none.
  int alt = -1;
};

struct Stratum {
  std::vector<int> rels;        // derived relations of this stratum
  std::vector<int> base_plans;  // plan ids run in round 1
  std::vector<int> delta_plans; // plan ids run in rounds >= 2
  bool recursive = false;
};

struct Program {
  std::vector<Relation> rels;
  std::vector<Rule> rules;
  std::vector<Stratum> strata;
  std::vector<Plan> plans;
  std::vector<IndexSpec> indexes;
  int max_cols = 0;             // widest packed table (columns, excluding the sample)
  uint32_t max_const = 0;       // largest constant of the program (a lower bound of the id domain)
  int find(const std::string& name) const;
};

// Returns 0 on success, else 2 (parse error) or 3 (unsupported) with `err` set.
int parse_and_plan(const char* text, bool frozen_tags, bool diff_lineage, Program& out, std::string& err);

}  // namespace dlfix
