"""Pins of the oracle's differentiable max-min semiring (tags are pairs of a
probability and the input fact it comes from; x keeps the smaller value, +
the larger one, equal values keep the smaller fact number), computed here
from the mathematics:

* values: widest-path closure (Floyd-Warshall over (max, min)), exact;
* facts: the tag of path(x, z) comes from the smallest-numbered edge e = (u, w)
  whose probability equals the widest value v and that lies on an x -> z walk
  of edges of probability >= v (u reachable from x, z from w, both through
  such edges, or u = x / w = z);
* gradient: 1 for that edge, 0 for all others; central differences of the
  oracle's own values agree;
* the pair operations' laws (+ and x commutative and associative, +
  idempotent, identities).
"""
import itertools

import numpy as np
import pytest

TC = ".input edge/2\npath(x, y) :- edge(x, y).\npath(x, z) :- edge(x, y), path(y, z).\n"


def run(oracle, src, dst, p):
    o = oracle.Oracle(TC, "diff_maxmin")
    o.add_facts("edge", [src, dst], p)
    return o.run()


def widest(n, src, dst, p):
    W = np.zeros((n, n))
    for a, b, q in zip(src, dst, p):
        W[a, b] = max(W[a, b], float(q))
    for k in range(n):
        W = np.maximum(W, np.minimum(W[:, k:k + 1], W[k:k + 1, :]))
    return W


def reach_at_least(n, src, dst, p, v):
    """R[a, b]: b reachable from a (0 or more edges) through edges >= v."""
    keep = np.asarray(p, np.float64) >= v
    A = np.zeros((n, n), bool)
    A[src[keep], dst[keep]] = True
    # reflexive-transitive closure of A: (I | A) squared until it covers n steps
    M = np.eye(n, dtype=bool) | A
    for _ in range(int(np.ceil(np.log2(max(n, 2)))) + 1):
        M = M | ((M.astype(np.int64) @ M.astype(np.int64)) > 0)
    return M


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_values_and_facts(oracle, synth, seed):
    n, m = 30, 70
    src, dst, p = synth.er_graph(seed, n, m, weights=True)
    o = run(oracle, src, dst, p)
    r = o.read("path")
    fid = o.fid("path")
    W = widest(n, src, dst, p)
    cols = r["cols"]
    assert set(map(tuple, cols.tolist())) == set(zip(*np.nonzero(W > 0)))
    assert np.array_equal(r["value"], W[cols[:, 0], cols[:, 1]])
    for (x, z), f, v in zip(cols.tolist(), fid.tolist(), r["value"].tolist()):
        M = reach_at_least(n, src, dst, p, v)
        best = None
        for e in range(m):
            if float(p[e]) == v and M[x, src[e]] and M[dst[e], z]:
                best = e
                break
        assert f == best, (x, z)


def test_gradient_is_the_bottleneck_fact(oracle, synth):
    n, m = 25, 60
    src, dst, p = synth.er_graph(4, n, m, weights=True)
    o = run(oracle, src, dst, p)
    r = o.read("path")
    g = synth.normal_grads(1, r["cols"].shape[0]).astype(np.float64)
    o.backward("path", g)
    grad = o.grad("edge", m)
    want = np.zeros(m)
    np.add.at(want, o.fid("path"), g)
    assert np.array_equal(grad, want)
    # central differences of g . values on a few edges
    rng = np.random.default_rng(0)
    h = 1e-5
    for e in rng.choice(m, 8, replace=False):
        vals = []
        for sgn in (1, -1):
            p2 = p.copy()
            p2[e] = np.float32(p2[e] + sgn * h)
            vals.append((float(g @ run(oracle, src, dst, p2).read("path")["value"]), float(p2[e])))
        fd = (vals[0][0] - vals[1][0]) / (vals[0][1] - vals[1][1])
        assert fd == pytest.approx(grad[e], abs=1e-6), e


def test_pair_laws(oracle):
    vals = [(0.25, 3), (0.5, 1), (0.5, 2), (0.75, 0), (0.25, 0)]
    op = oracle.vid_op
    for a, b in itertools.product(vals, vals):
        for o in ("plus", "times"):
            assert op(o, a, b) == op(o, b, a)
        assert op("plus", a, a) == a and op("times", a, a) == a
    for a, b, c in itertools.product(vals, vals, vals):
        for o in ("plus", "times"):
            assert op(o, op(o, a, b), c) == op(o, a, op(o, b, c))
    for a in vals:
        assert op("plus", a, (0.0, 2**32 - 1)) == a   # zero: nothing derived
        assert op("times", a, (1.0, 2**32 - 1)) == a  # one: a certain fact
