"""Seeded synthetic inputs for the semiring fixpoint engine and its CPU oracle.

This module only draws random relations; it holds none of the method's
arithmetic (no join, no tag algebra), so both the HIP path and the oracle may
take their inputs from it without sharing any computation.  It imports nothing
from the rest of the package.

Every workload stands in for a dataset the paper measures but that is not
available here: Erdos-Renyi graphs for the SNAP transitive-closure graphs
(Sec. 6.1, transitive closure), k x k grids for the Pathfinder lattice
(Sec. 2), Zipf-skewed points-to facts for the CSPA inputs (Sec. 6.1), and small
random relational scenes for CLUTRR-style top-k proof tasks (Sec. 6.1).
"""
from __future__ import annotations

import numpy as np

TC_PROGRAM = """
.input edge/2
.output path/2
path(x, y) :- edge(x, y).
path(x, z) :- edge(x, y), path(y, z).
"""

# Same Generation (the paper's second discrete workload), with its selection
SG_PROGRAM = """
.input edge/2
.output sg/2
sg(x, y) :- edge(p, x), edge(p, y), x != y.
sg(x, y) :- edge(a, x), sg(a, b), edge(b, y).
"""

# The motivating program: reachability between the endpoints of a grid
PATHFINDER_PROGRAM = """
.input edge/2
.input is_endpoint/1
.output endpoints_connected/0
path(x, y) :- edge(x, y).
path(x, z) :- path(x, y), edge(y, z).
endpoints_connected() :- is_endpoint(x), is_endpoint(y), path(x, y), x != y.
"""

ANDERSEN_PROGRAM = """
.input addr/2
.input assign/2
.input load/2
.input store/2
.output pt/2
pt(v, o) :- addr(v, o).
pt(v, o) :- assign(v, w), pt(w, o).
pt(v, o) :- load(v, p), pt(p, q), pt(q, o).
pt(q, o) :- store(p, w), pt(p, q), pt(w, o).
"""

TOPK_PROGRAM = """
.input u0/1
.input u1/1
.input u2/1
.input u3/1
.input u4/1
.input u5/1
.input u6/1
.input u7/1
.input r0/2
.input r1/2
.input r2/2
.input r3/2
.output q/2
.output reach/2
q(a, b) :- u0(a), r0(a, b), u1(b).
reach(a, b) :- r1(a, b).
reach(a, c) :- r1(a, b), reach(b, c).
"""


def _distinct_pairs(rng: np.random.Generator, n: int, m: int,
                    lo: int = 0) -> tuple[np.ndarray, np.ndarray]:
    """m distinct ordered pairs (u, v), u != v, uniform over [lo, lo+n)^2,
    in the order they were first drawn (rejection sampling)."""
    if m > n * (n - 1):
        raise ValueError("too many pairs requested")
    keys = np.empty(0, dtype=np.int64)
    while keys.size < m:
        want = max(64, 2 * (m - keys.size))
        u = rng.integers(0, n, size=want)
        v = rng.integers(0, n, size=want)
        k = (u * n + v)[u != v]
        keys = np.concatenate([keys, k])
        _, first = np.unique(keys, return_index=True)
        keys = keys[np.sort(first)]
    keys = keys[:m]
    return (keys // n + lo).astype(np.uint32), (keys % n + lo).astype(np.uint32)


def er_graph(seed: int, n: int, m: int, weights: bool = False):
    """Directed G(n, m): m distinct ordered pairs, no self loops.

    Returns (src, dst, p) with p = float32 U(0.1, 0.9) when `weights`, else None.
    """
    rng = np.random.default_rng(seed)
    src, dst = _distinct_pairs(rng, n, m)
    p = rng.uniform(0.1, 0.9, size=m).astype(np.float32) if weights else None
    return src, dst, p


def unit_prob(rng: np.random.Generator, size) -> np.ndarray:
    """float32 probabilities in (0, 1) on a 2^-24 lattice (never 0, never 1)."""
    return (rng.integers(1, 1 << 24, size=size).astype(np.float64)
            * (1.0 / (1 << 24))).astype(np.float32)


def grid_edges(k: int) -> tuple[np.ndarray, np.ndarray]:
    """Both directions between 4-neighbours of a k x k grid, row-major cell ids."""
    src, dst = [], []
    for r in range(k):
        for c in range(k):
            a = r * k + c
            if c + 1 < k:
                src += [a, a + 1]
                dst += [a + 1, a]
            if r + 1 < k:
                src += [a, a + k]
                dst += [a + k, a]
    return np.asarray(src, np.uint32), np.asarray(dst, np.uint32)


def grid_batch(seed: int, samples: int = 512, kmin: int = 5, kmax: int = 30):
    """Batched k x k grids, k ~ U{kmin..kmax}; edge probabilities in (0, 1).

    Returns dict(sample, src, dst, p, ks, labels): edges of all samples
    concatenated in sample order, plus a seeded Bernoulli(0.5) label per sample.
    """
    rng = np.random.default_rng(seed)
    ks = rng.integers(kmin, kmax + 1, size=samples)
    ss, us, vs = [], [], []
    for s, k in enumerate(ks):
        u, v = grid_edges(int(k))
        ss.append(np.full(u.size, s, np.uint32))
        us.append(u)
        vs.append(v)
    sample = np.concatenate(ss)
    p = unit_prob(rng, sample.size)
    labels = (rng.random(samples) < 0.5).astype(np.float32)
    return dict(sample=sample, src=np.concatenate(us), dst=np.concatenate(vs),
                p=p, ks=ks.astype(np.int64), labels=labels)


def zipf_ids(rng: np.random.Generator, v: int, size: int, s: float,
             perm: np.ndarray) -> np.ndarray:
    """Bounded Zipf: P(r) ~ r^-s over ranks 1..v, mapped through `perm`."""
    w = np.arange(1, v + 1, dtype=np.float64) ** (-s)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    r = np.searchsorted(cdf, rng.random(size), side="right")
    r = np.minimum(r, v - 1)
    return perm[r]


def _zipf_relation(rng, v, count, s, perm):
    keys = np.empty(0, dtype=np.int64)
    while keys.size < count:
        want = max(1024, 2 * (count - keys.size))
        a = zipf_ids(rng, v, want, s, perm).astype(np.int64)
        b = zipf_ids(rng, v, want, s, perm).astype(np.int64)
        k = (a * v + b)[a != b]
        keys = np.concatenate([keys, k])
        _, first = np.unique(keys, return_index=True)
        keys = keys[np.sort(first)]
    keys = keys[:count]
    return (keys // v).astype(np.uint32), (keys % v).astype(np.uint32)


def andersen(seed: int, v: int = 100_000, n_addr: int = 50_000,
             n_assign: int = 300_000, n_load: int = 40_000,
             n_store: int = 40_000, s: float = 1.2):
    """Points-to facts with Zipf(s) endpoints over one id domain of size v.

    Each relation has exactly its count of distinct tuples and no self pairs.
    Returns dict name -> (col0, col1).
    """
    rng = np.random.default_rng(seed)
    perm = rng.permutation(v).astype(np.int64)
    out = {}
    for name, cnt in (("addr", n_addr), ("assign", n_assign),
                      ("load", n_load), ("store", n_store)):
        out[name] = _zipf_relation(rng, v, cnt, s, perm)
    return out


def topk_scenes(seed: int, samples: int = 256, nmin: int = 10, nmax: int = 40,
                unary: int = 8, binary: int = 4, per_unary: int = 4,
                per_binary: int = 8):
    """Batched relational scenes for the top-k proof workload.

    Per sample: n ~ U{nmin..nmax} objects; each unary relation u_i gets
    `per_unary` distinct objects, each binary relation r_i gets `per_binary`
    distinct ordered pairs (a != b).  Probabilities in (0, 1).  Facts are listed
    relation by relation (u0..u7 then r0..r3), sample by sample inside each
    relation.  Returns dict name -> (sample, cols..., p) plus 'ns'.
    """
    rng = np.random.default_rng(seed)
    ns = rng.integers(nmin, nmax + 1, size=samples)
    per = {f"u{i}": ([], [], []) for i in range(unary)}
    per.update({f"r{i}": ([], [], [], []) for i in range(binary)})
    for s, n in enumerate(ns):
        n = int(n)
        for i in range(unary):
            objs = rng.choice(n, size=per_unary, replace=False).astype(np.uint32)
            per[f"u{i}"][0].append(np.full(per_unary, s, np.uint32))
            per[f"u{i}"][1].append(objs)
            per[f"u{i}"][2].append(unit_prob(rng, per_unary))
        for i in range(binary):
            a, b = _distinct_pairs(rng, n, per_binary)
            per[f"r{i}"][0].append(np.full(per_binary, s, np.uint32))
            per[f"r{i}"][1].append(a)
            per[f"r{i}"][2].append(b)
            per[f"r{i}"][3].append(unit_prob(rng, per_binary))
    out = {name: tuple(np.concatenate(c) for c in cols) for name, cols in per.items()}
    out["ns"] = ns.astype(np.int64)
    return out


def normal_grads(seed: int, n: int) -> np.ndarray:
    """Seeded N(0, 1) output gradients (float32)."""
    return np.random.default_rng(seed).standard_normal(n).astype(np.float32)
