"""Pins of the oracle's expression evaluation (comparisons in rule bodies,
arithmetic head terms, constants in atoms, nullary relations) against closed
forms computed here from the mathematics, not from the oracle:

* Same Generation with its x != y selection on random out-trees: two distinct
  nodes at the same depth >= 1 are of the same generation, by exactly one
  derivation, whose tag is the product of the edges on the two paths up to
  their lowest common ancestor (one edge pair per level); on general graphs,
  the union over k of (E^T)^k S0 E^k in the boolean and (max, min) matrix
  algebras, with its first round.
* Walks of an exact length with an arithmetic hop counter and a bound: the
  tag of walk(x, z, d) is entry (x, z) of the d-th semiring matrix power of
  the edge matrix (add-mult: clamped at 1 after every product, because every
  walk of length d is derived in round d).
* Constants in atoms and nullary heads: reachability from node 0 by breadth
  first search, presence of a cycle.
* Arithmetic filters, repeated variables and division by zero: brute force
  over the edge list.
"""
import numpy as np
import pytest

SG = """
.input edge/2
sg(x, y) :- edge(p, x), edge(p, y), x != y.
sg(x, y) :- edge(a, x), sg(a, b), edge(b, y).
"""

WALK = """
.input edge/2
walk(x, y, 1) :- edge(x, y).
walk(x, z, d + 1) :- walk(x, y, d), edge(y, z), d < {L}.
"""

REACH = """
.input edge/2
path(x, y) :- edge(x, y).
path(x, z) :- edge(x, y), path(y, z).
from0(y) :- path(0, y).
cyclic() :- path(x, x).
"""

FILTERS = """
.input edge/2
loop(x) :- edge(x, x).
even_big(x, y) :- edge(x, y), x + y > 10, x % 2 == 0.
ratio(x, y / x, y - x) :- edge(x, y), y >= x.
dbl(x, y, x * 3) :- edge(x, y), x * 2 <= y, y < 11.
"""

PATHFINDER = """
.input edge/2
.input is_endpoint/1
path(x, y) :- edge(x, y).
path(x, z) :- path(x, y), edge(y, z).
endpoints_connected() :- is_endpoint(x), is_endpoint(y), path(x, y), x != y.
"""


def run(oracle, program, sr, facts):
    o = oracle.Oracle(program, sr)
    for rel, (cols, tags) in facts.items():
        o.add_facts(rel, cols, None if sr == "bool" else tags)
    return o.run()


def random_tree(seed, n):
    rng = np.random.default_rng(seed)
    parent = np.array([-1] + [int(rng.integers(0, i)) for i in range(1, n)])
    p = rng.uniform(0.1, 0.9, n).astype(np.float32)  # p[i]: edge parent[i] -> i
    return parent, p


OTIMES = {"bool": lambda a, b: 1.0, "maxmin": min, "minplus": lambda a, b: a + b,
          "addmult": lambda a, b: a * b}


@pytest.mark.parametrize("sr", ["bool", "maxmin", "minplus", "addmult"])
@pytest.mark.parametrize("seed", [1, 2, 3])
def test_same_generation_on_trees(oracle, sr, seed):
    n = 60
    parent, p = random_tree(seed, n)
    src = parent[1:].astype(np.uint32)
    dst = np.arange(1, n, dtype=np.uint32)
    o = run(oracle, SG, sr, {"edge": ([src, dst], p[1:])})
    depth = np.zeros(n, int)
    for i in range(1, n):
        depth[i] = depth[parent[i]] + 1
    want = {}
    for x in range(1, n):
        for y in range(1, n):
            if x == y or depth[x] != depth[y]:
                continue
            a, b, t = x, y, None
            while a != b:  # climb both paths one level at a time
                for e in (a, b):
                    t = float(p[e]) if t is None else OTIMES[sr](t, float(p[e]))
                a, b = parent[a], parent[b]
            want[(x, y)] = t
    r = o.read("sg")
    got = {(int(a), int(b)): v for (a, b), v in zip(r["cols"], r["value"])}
    assert set(got) == set(want)
    if sr != "bool":
        for k, v in want.items():
            assert got[k] == pytest.approx(v, rel=1e-12), k


def mm_product(X, Y):
    """(max, min) matrix product."""
    return np.max(np.minimum(X[:, :, None], Y[None, :, :]), axis=1)


@pytest.mark.parametrize("sr", ["bool", "maxmin"])
@pytest.mark.parametrize("seed", [1, 2])
def test_same_generation_matrix_form(oracle, synth, sr, seed):
    """Same Generation on general (cyclic) graphs in matrix form: with E the
    edge matrix and S0 the pairs of distinct children of one parent, the
    relation is the union over k >= 0 of (E^T)^k S0 E^k, products in the
    semiring (boolean, or (max, min) with the value the best over k), and a
    pair is first derived in round k + 1 for the smallest such k."""
    n, m = 60, 150
    src, dst, p = synth.er_graph(seed, n, m, weights=True)
    E = np.zeros((n, n))
    E[src, dst] = p.astype(np.float64) if sr == "maxmin" else 1.0
    S0 = np.max(np.minimum(E[:, :, None], E[:, None, :]), axis=0)  # over the parent
    np.fill_diagonal(S0, 0.0)
    best, first = S0.copy(), np.where(S0 > 0, 1, 0)
    X, k = S0, 0
    while True:
        k += 1
        X = mm_product(mm_product(E.T, X), E)
        first = np.where((first == 0) & (X > 0), k + 1, first)
        if np.all(X <= best):  # then so is every later term: the products are monotone
            break
        best = np.maximum(best, X)
    o = run(oracle, SG, sr, {"edge": ([src, dst], p)})
    r = o.read("sg")
    want = np.argwhere(best > 0)
    assert want.shape[0] > 100
    assert np.array_equal(r["cols"], want.astype(np.uint32))
    if sr == "maxmin":
        assert np.array_equal(r["value"], best[want[:, 0], want[:, 1]])
    else:
        assert np.array_equal(r["round"], first[want[:, 0], want[:, 1]].astype(np.int32))


def semiring_power(P, present, d, sr):
    """d-th power of the edge matrix in the semiring (absent = semiring zero)."""
    T, TP = P.copy(), present.copy()
    for _ in range(d - 1):
        if sr == "addmult":
            T2 = np.minimum(1.0, T @ P)
        elif sr == "maxmin":
            T2 = np.max(np.minimum(T[:, :, None], P[None, :, :]), axis=1)
        elif sr == "minplus":
            T2 = np.min(T[:, :, None] + P[None, :, :], axis=1)
        else:
            T2 = ((TP.astype(int) @ present.astype(int)) > 0).astype(float)
        TP = (TP.astype(int) @ present.astype(int)) > 0
        T = T2
    return T, TP


@pytest.mark.parametrize("sr", ["bool", "maxmin", "minplus", "addmult"])
def test_walks_of_exact_length(oracle, synth, sr):
    n, m, L = 40, 90, 4
    src, dst, p = synth.er_graph(4, n, m, weights=True)
    p = (p * 0.3).astype(np.float32)  # keep add-mult sums mostly below the clamp
    o = run(oracle, WALK.format(L=L), sr, {"edge": ([src, dst], p)})
    r = o.read("walk")
    present = np.zeros((n, n), bool)
    present[src, dst] = True
    zero = {"addmult": 0.0, "maxmin": 0.0, "minplus": np.inf, "bool": 0.0}[sr]
    P = np.full((n, n), zero)
    P[src, dst] = p.astype(np.float64)
    got = {(int(a), int(b), int(c)): v for (a, b, c), v in zip(r["cols"], r["value"])}
    want = {}
    for d in range(1, L + 1):
        T, TP = semiring_power(P, present, d, sr)
        for x, z in zip(*np.nonzero(TP)):
            want[(int(x), int(z), d)] = T[x, z]
    assert set(got) == set(want)
    if sr != "bool":
        for k, v in want.items():
            assert got[k] == pytest.approx(v, rel=1e-12), k


def test_constants_and_nullary(oracle, synth):
    n, m = 30, 45
    src, dst, p = synth.er_graph(5, n, m, weights=True)
    o = run(oracle, REACH, "maxmin", {"edge": ([src, dst], p)})
    adj = [[] for _ in range(n)]
    for a, b in zip(src, dst):
        adj[a].append(int(b))
    seen, stack = set(), list(adj[0])
    while stack:
        v = stack.pop()
        if v not in seen:
            seen.add(v)
            stack.extend(adj[v])
    assert sorted(int(y) for y in o.read("from0")["cols"][:, 0]) == sorted(seen)
    # widest paths with >= 1 edge (Floyd-Warshall over max-min); the nullary
    # head holds the best cycle tag: max over x of W[x, x]
    W = np.zeros((n, n))
    W[src, dst] = p
    for k in range(n):
        W = np.maximum(W, np.minimum(W[:, k:k + 1], W[k:k + 1, :]))
    c = o.read("cyclic")
    if W.diagonal().max() > 0:
        assert c["cols"].shape == (1, 0)
        assert c["value"][0] == W.diagonal().max()
    else:
        assert c["cols"].shape[0] == 0
    f0 = o.read("from0")
    assert np.array_equal(f0["value"], W[0, f0["cols"][:, 0]])


def test_filters_repeats_and_division(oracle):
    rng = np.random.default_rng(6)
    src = rng.integers(0, 12, 80).astype(np.uint32)
    dst = rng.integers(0, 12, 80).astype(np.uint32)
    o = run(oracle, FILTERS, "bool", {"edge": ([src, dst], None)})
    pairs = set(zip(src.tolist(), dst.tolist()))
    assert sorted(o.read("loop")["cols"][:, 0].tolist()) == sorted({a for a, b in pairs if a == b})
    want = sorted((a, b) for a, b in pairs if a + b > 10 and a % 2 == 0)
    assert sorted(map(tuple, o.read("even_big")["cols"].tolist())) == want
    want = sorted({(a, b // a, b - a) for a, b in pairs if b >= a and a != 0})  # x = 0: divided by zero
    assert sorted(map(tuple, o.read("ratio")["cols"].tolist())) == want
    want = sorted({(a, b, 3 * a) for a, b in pairs if 2 * a <= b < 11})
    assert sorted(map(tuple, o.read("dbl")["cols"].tolist())) == want


@pytest.mark.parametrize("seed", [1, 2, 3, 4])
def test_pathfinder_endpoints(oracle, synth, seed):
    """The motivating program's nullary query under bool tags: true iff two
    distinct endpoints are connected."""
    n = 25
    src, dst, _ = synth.er_graph(seed, n, 30, weights=True)
    rng = np.random.default_rng(seed)
    ends = rng.choice(n, 3, replace=False).astype(np.uint32)
    o = run(oracle, PATHFINDER, "bool", {"edge": ([src, dst], None), "is_endpoint": ([ends], None)})
    R = np.zeros((n, n), bool)
    R[src, dst] = True
    for k in range(n):
        R |= R[:, k:k + 1] & R[k:k + 1, :]
    want = any(R[x, y] for x in ends for y in ends if x != y)
    assert o.size("endpoints_connected") == int(want)


def test_unbound_comparison_variable_is_rejected(oracle):
    with pytest.raises(ValueError):
        oracle.Oracle(".input edge/2\nq(x) :- edge(x, y), z > 1.\n", "bool")
    with pytest.raises(ValueError):
        oracle.Oracle(".input edge/2\nq(x, w + 1) :- edge(x, y).\n", "bool")
