"""Semiring laws of the oracle's tag algebra on random tags (Sec. 3.1: a
provenance semiring is (T, 0, 1, +, x)); top-k lists keep the k most likely
distinct proofs."""
import itertools

import numpy as np
import pytest

SCALAR = ["maxmin", "minplus", "addmult"]


@pytest.mark.parametrize("sr", SCALAR)
def test_scalar_laws(oracle, sr):
    rng = np.random.default_rng(0)
    vals = [float(np.float32(x)) for x in rng.uniform(0.05, 0.95, 8)]
    plus = lambda a, b: oracle.scalar_op(sr, "plus", a, b)
    times = lambda a, b: oracle.scalar_op(sr, "times", a, b)
    zero, one = oracle.scalar_identity(sr, "zero"), oracle.scalar_identity(sr, "one")
    for a, b in itertools.product(vals, vals):
        assert plus(a, b) == plus(b, a)
        assert times(a, b) == times(b, a)
        assert plus(a, zero) == a
        assert times(a, one) == a
        assert times(a, zero) == zero
    for a, b, c in itertools.product(vals[:5], vals[:5], vals[:5]):
        assert plus(plus(a, b), c) == pytest.approx(plus(a, plus(b, c)), rel=1e-15)
        assert times(times(a, b), c) == pytest.approx(times(a, times(b, c)), rel=1e-15)
        if sr != "addmult":  # distributivity holds exactly for the lattice/tropical semirings
            assert times(a, plus(b, c)) == pytest.approx(plus(times(a, b), times(a, c)), rel=1e-15)
    idem = sr != "addmult"
    for a in vals:
        assert (plus(a, a) == a) == idem
    if sr == "addmult":
        assert plus(0.7, 0.6) == 1.0  # + saturates at 1


def random_list(rng, k, nfacts=10):
    n = int(rng.integers(0, k + 1))
    out = set()
    while len(out) < n:
        out.add(int(rng.integers(1, 1 << nfacts)))
    return sorted(out)


def brute_best(cands, q, k):
    def prob(b):
        acc = np.float32(1.0)
        for i in range(64):
            if b >> i & 1:
                acc = np.float32(acc * np.float32(q[i]))
        return acc
    ranked = sorted(set(cands), key=lambda b: (-prob(b), b))[:k]
    return ranked


@pytest.mark.parametrize("k", [1, 2, 3])
def test_topk_ops_are_best_k_of_union(oracle, k):
    rng = np.random.default_rng(k)
    q = np.zeros(64, np.float32)
    q[:10] = rng.uniform(0.05, 0.95, 10).astype(np.float32)
    for _ in range(200):
        a, b = random_list(rng, k), random_list(rng, k)
        bits, probs = oracle.topk_op(k, "plus", a, b, q)
        assert bits == brute_best(a + b, q, k)
        assert all(probs[i] >= probs[i + 1] for i in range(len(probs) - 1))
        bits, _ = oracle.topk_op(k, "times", a, b, q)
        assert bits == brute_best([x | y for x in a for y in b], q, k)


def test_topk_plus_laws(oracle):
    rng = np.random.default_rng(9)
    q = np.zeros(64, np.float32)
    q[:10] = rng.uniform(0.05, 0.95, 10).astype(np.float32)
    k = 3
    P = lambda a, b: oracle.topk_op(k, "plus", a, b, q)[0]
    T = lambda a, b: oracle.topk_op(k, "times", a, b, q)[0]
    for _ in range(100):
        a, b, c = random_list(rng, k), random_list(rng, k), random_list(rng, k)
        assert P(a, b) == P(b, a)
        assert P(P(a, b), c) == P(a, P(b, c))      # best-k of a union: associative
        if a:
            assert P(P(a, []), P(a, [])) == P(a, [])  # idempotent
        assert T(a, b) == T(b, a)
        assert T(a, [0]) == P(a, [])               # {} (the empty proof) is the unit of x
        assert T(a, []) == []                      # the empty list is absorbing
