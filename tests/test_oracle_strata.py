"""Pins of the oracle's stratum order (Algorithm 1: strata are evaluated one
after the other, each to its own fixpoint, in dependency order).

The programs below list their rules (and declare their outputs) in the
reverse of the dependency order, so an evaluator that ran strata in order of
first mention, or that iterated every rule together, would read relations of
an unfinished lower stratum.  Expected values come from closed forms computed
here with numpy/scipy, not from the oracle.
"""
import numpy as np
import pytest
from scipy.sparse import csr_matrix
from scipy.sparse.csgraph import dijkstra

from test_oracle_pins import grid_closed_form

# top is the transitive closure of hop, hop = (>= 1-edge closure of edge) o edge
CHAIN = """
.input edge/2
.output top/2
.output hop/2
top(x, z) :- hop(x, y), top(y, z).
top(x, y) :- hop(x, y).
hop(x, z) :- path(x, y), edge(y, z).
path(x, y) :- edge(x, y).
path(x, z) :- edge(x, y), path(y, z).
"""

# a non-recursive stratum over a recursive one
HOP = """
.input edge/2
.output hop/2
hop(x, z) :- path(x, y), edge(y, z).
path(x, y) :- edge(x, y).
path(x, z) :- edge(x, y), path(y, z).
"""


def run(oracle, program, sr, src, dst, p):
    o = oracle.Oracle(program, sr)
    o.add_facts("edge", [src, dst], p)
    return o.run()


def widest_closure(W):
    """Bottleneck (max-min) closure over walks of >= 1 step (Floyd-Warshall)."""
    W = W.copy()
    for k in range(W.shape[0]):
        W = np.maximum(W, np.minimum(W[:, k : k + 1], W[k : k + 1, :]))
    return W


def maxmin_compose(A, B):
    """C[x, z] = max_y min(A[x, y], B[y, z])."""
    return np.max(np.minimum(A[:, :, None], B[None, :, :]), axis=1)


def minplus_closure(W):
    """Shortest walks of >= 1 step (inf = no walk), via scipy Dijkstra."""
    n = W.shape[0]
    fin = np.isfinite(W)
    A = csr_matrix((W[fin], np.nonzero(fin)), shape=(n, n))
    d = dijkstra(A)  # d[z, z] = 0 (empty walk)
    # first step, then any walk
    return np.min(W[:, :, None] + d[None, :, :], axis=1)


def check_matrix(res, M, absent, exact):
    want = np.argwhere(M != absent)
    assert np.array_equal(res["cols"], want.astype(np.uint32))
    if exact:
        assert np.array_equal(res["value"], M[want[:, 0], want[:, 1]])
    else:
        np.testing.assert_allclose(res["value"], M[want[:, 0], want[:, 1]], rtol=1e-12)


@pytest.mark.parametrize("seed", [1, 2])
def test_chain_maxmin_vs_closed_form(oracle, synth, seed):
    n = 60
    src, dst, p = synth.er_graph(seed, n, 150, weights=True)
    E = np.zeros((n, n))
    E[src, dst] = p.astype(np.float64)
    W = widest_closure(E)
    H = maxmin_compose(W, E)
    T = widest_closure(H)
    o = run(oracle, CHAIN, "maxmin", src, dst, p)
    check_matrix(o.read("path"), W, 0.0, exact=True)
    check_matrix(o.read("hop"), H, 0.0, exact=True)
    check_matrix(o.read("top"), T, 0.0, exact=True)
    # bool: the same supports
    ob = run(oracle, CHAIN, "bool", src, dst, None)
    for rel, M in (("path", W), ("hop", H), ("top", T)):
        assert np.array_equal(ob.read(rel)["cols"], np.argwhere(M > 0).astype(np.uint32)), rel


def test_chain_minplus_vs_dijkstra(oracle, synth):
    n = 60
    src, dst, p = synth.er_graph(3, n, 150, weights=True)
    E = np.full((n, n), np.inf)
    E[src, dst] = p.astype(np.float64)
    D = minplus_closure(E)
    H = np.min(D[:, :, None] + E[None, :, :], axis=1)
    T = minplus_closure(H)
    o = run(oracle, CHAIN, "minplus", src, dst, p)
    check_matrix(o.read("path"), D, np.inf, exact=False)
    check_matrix(o.read("hop"), H, np.inf, exact=False)
    check_matrix(o.read("top"), T, np.inf, exact=False)


@pytest.mark.parametrize("k", [3, 4])
def test_hop_over_grid_addmult_closed_form(oracle, synth, k):
    """Frozen add-mult: hop is a stratum of its own, evaluated once on the
    finished path relation, so every neighbour y of z contributes:
    hop(x, z) = min(1, sum over edges (y, z) of path(x, y) p(y, z)).
    Evaluating hop alongside path would freeze it at its first (shortest)
    derivations instead."""
    rng = np.random.default_rng(10 + k)
    src, dst = synth.grid_edges(k)
    p = synth.unit_prob(rng, src.size)
    path = grid_closed_form(k, src, dst, p)  # every pair: grids are strongly connected
    n = k * k
    want = {}
    for x in range(n):
        for z in range(n):
            s = sum(path[(x, int(y))] * float(q) for y, zz, q in zip(src, dst, p) if zz == z)
            want[(x, z)] = min(1.0, s)
    o = run(oracle, HOP, "addmult", src, dst, p)
    r = o.read("hop")
    got = {(int(a), int(b)): v for (a, b), v in zip(r["cols"], r["value"])}
    assert sorted(got) == sorted(want)
    for key, v in want.items():
        assert got[key] == pytest.approx(v, rel=1e-12), key
    # strata: path first (longest shortest walk 2(k-1) hops, plus the final
    # empty round), then hop (non-recursive: 2 rounds)
    assert lib_rounds(o) == [2 * (k - 1) + 1, 2]


def lib_rounds(o):
    from oracle import ref
    ns = ref.lib().ref_num_strata(o.h)
    return [o.rounds(s) for s in range(ns)]
