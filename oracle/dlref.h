/* CPU oracle for semiring Datalog fixpoints -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, obviously-correct reference used by the tests, the smoke check
 * and the CPU-baseline leg of the benchmark.  The product (HIP) path never
 * links, includes or calls anything here, and nothing here includes the
 * product's headers.
 *
 * What it computes (the paper's method, restated):
 *   - Programs are positive Datalog rules grouped into strata (SCCs of the
 *     predicate dependency graph, topological order); strata run one after the
 *     other and each one iterates to a fixpoint (Appendix B, Algorithm 1).
 *   - Every fact carries a provenance tag from a semiring (T, 0, 1, +, x)
 *     (Sec. 3.1 "Provenance Semirings", Sec. 3.5).  A derivation's value is the
 *     x-product of its body tags left to right; a head's candidate is the
 *     +-sum of its derivations' values.
 *   - Rounds are naive and Jacobi: every derivation of a round reads the tags
 *     at the end of the previous round.  Round 1 of a stratum fires every rule
 *     on everything known so far (recent = F_T in Algorithm 1).
 *   - Idempotent semirings (bool, max-min, min-plus, top-k) converge: a tuple's
 *     tag absorbs every derivation (t <- t + cand).  Add-mult is frozen at
 *     discovery: the tag is the sum over the derivations of the discovery
 *     round, later derivations are ignored.  A stratum stops at the first
 *     round with no new tuple and no changed tag.
 */
#ifndef DLREF_H
#define DLREF_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  REF_BOOL = 0,
  REF_MAXMIN = 1,
  REF_MINPLUS = 2,
  REF_ADDMULT = 3,
  REF_DIFF_ADDMULT = 4,
  REF_TOPK = 5,
  REF_DIFF_TOPK = 6,
  REF_DIFF_MAXMIN = 7  /* max-min with the input fact its value comes from (see ref_read_fid) */
};

typedef struct ref_engine ref_engine;

/* Parse `program`; k is the proof count for the top-k semirings (1..3). */
int ref_create(const char* program, int semiring, int k, int batched,
               ref_engine** out, char* err, size_t errlen);
/* cols is row-major n x arity; tags are float32 (NULL for bool); sample_ids
 * NULL unless batched.  Facts are copied. */
int ref_add_facts(ref_engine*, const char* rel, size_t n,
                  const uint32_t* sample_ids, const uint32_t* cols,
                  const float* tags);
int ref_run(ref_engine*);
long ref_size(ref_engine*, const char* rel);
/* Rounds of the given stratum, maximum over samples (stratum index in
 * evaluation order).  Returns -1 if out of range. */
int ref_rounds(ref_engine*, int stratum);
int ref_num_strata(ref_engine*);
/* Canonical (sample, col0, col1, ...) order.  Any output pointer may be NULL.
 * value: f64 tag (bool: 1.0).  Top-k: cnt[n], bits[n*3], p[n*3] (float32
 * canonical proof probabilities), prob[n] = inclusion-exclusion probability. */
int ref_read(ref_engine*, const char* rel, uint32_t* sample_ids, uint32_t* cols,
             double* value, int32_t* cnt, uint64_t* bits, float* p,
             double* prob, int32_t* round_found);
/* Top-k proofs as full fact sets (up to 256 probabilistic facts per sample,
 * Sec. 3.5 top-k proofs): word w of proof j of tuple i at
 * bits[(i*3 + j)*4 + w], fact f at bit f % 64 of word f / 64 (ref_read's
 * `bits` holds word 0 only). */
int ref_read_bits(ref_engine*, const char* rel, uint64_t* bits);
/* Differentiable max-min: the input fact (numbered 0, 1, ... over all
 * ref_add_facts calls in order) whose probability each tuple's tag equals;
 * its derivative with respect to that probability is 1, to all others 0.
 * Tags are (value, fact): x keeps the smaller value, + the larger one, and
 * equal values keep the smaller fact number. */
int ref_read_fid(ref_engine*, const char* rel, uint32_t* fid);
/* The pair operations of differentiable max-min (op 0 = plus, 1 = times). */
int ref_vid_op(int op, double av, uint32_t aid, double bv, uint32_t bid, double* ov, uint32_t* oid);

/* Reverse mode: seed d(loss)/d(tag) for every tuple of out_rel (canonical
 * order) and accumulate the input-fact gradients. */
int ref_backward(ref_engine*, const char* out_rel, const double* grad_out);
/* Input-fact gradients, aligned with the add order of in_rel. */
int ref_read_grad(ref_engine*, const char* in_rel, double* grad_in);
void ref_zero_grad(ref_engine*);
const char* ref_error(ref_engine*);
void ref_free(ref_engine*);

/* The oracle's tag algebra, exposed for the semiring-law tests.
 * Scalar semirings: *out = a (+ or x) b with op 0 = plus, 1 = times; the
 * top-k form takes proof lists (cnt, bits[3]) over facts with probabilities
 * q[64] and writes the resulting list.  zero/one return the identities. */
int ref_scalar_op(int semiring, int op, double a, double b, double* out);
int ref_scalar_identity(int semiring, int which, double* out);
int ref_topk_op(int k, int op, int acnt, const uint64_t* abits, int bcnt, const uint64_t* bbits,
                const float* q, int* ocnt, uint64_t* obits, float* oprob);

/* Single target column z of the transitive closure program
 *     path(x, y) :- edge(x, y).
 *     path(x, z) :- edge(x, y), path(y, z).
 * computed by the same naive Jacobi rounds restricted to tuples path(., z),
 * which only ever depend on other tuples of the same column.  Nodes are
 * 0..n-1.  Outputs per node x: present[x], tag[x] (f64), found[x] = round of
 * discovery; *rounds = rounds evaluated.  If grad_col != NULL (add-mult only),
 * grad_col[x] seeds d(loss)/d(tag of path(x,z)) and grad_edge[e] accumulates
 * the input gradients. */
int ref_tc_column(int n, size_t m, const uint32_t* src, const uint32_t* dst,
                  const float* w, int semiring, uint32_t z, uint8_t* present,
                  double* tag, int32_t* found, int32_t* rounds,
                  const double* grad_col, double* grad_edge);

/* Least solution of the four points-to rules
 *     pt(v,o) :- addr(v,o).           pt(v,o) :- assign(v,w), pt(w,o).
 *     pt(v,o) :- load(v,p), pt(p,q), pt(q,o).
 *     pt(q,o) :- store(p,w), pt(p,q), pt(w,o).
 * by worklist difference propagation.  Returns the handle of a result that
 * ref_pts_read copies out in (v, o) order. */
typedef struct ref_pts ref_pts;
ref_pts* ref_andersen(uint32_t nvars, size_t na, const uint32_t* addr,
                      size_t ns, const uint32_t* assign, size_t nl,
                      const uint32_t* load, size_t nst, const uint32_t* store);
long ref_pts_size(ref_pts*);
void ref_pts_read(ref_pts*, uint32_t* v, uint32_t* o);
void ref_pts_free(ref_pts*);

#ifdef __cplusplus
}
#endif
#endif
