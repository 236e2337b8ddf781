"""Pins of the oracle's top-k proofs over more than 64 probabilistic facts per
sample (proof sets of up to four 64-bit words, ordered as the integers they
spell), computed here from the mathematics:

* shift invariance: the same instance with D unused probabilistic facts
  numbered before its own (D = 70, 150) gives the same tuples, proof counts,
  proof probabilities and inclusion-exclusion probabilities, and proof sets
  equal to the unshifted ones times 2^D (the single-word oracle is pinned by
  brute force over possible worlds elsewhere);
* a 100-edge chain with a bypass: closed-form proofs, binary32 products in
  ascending fact order, the probability of the disjunction and its
  gradient;
* more than 256 probabilistic facts in a sample is refused.
"""
import numpy as np
import pytest

TC = """
.input pad/1
.input edge/2
path(x, y) :- edge(x, y).
path(x, z) :- path(x, y), edge(y, z).
"""


def as_int(words):
    return sum(int(w) << (64 * i) for i, w in enumerate(words))


def run(oracle, src, dst, p, pad=0, sr="topk", k=3):
    o = oracle.Oracle(TC, sr, k=k)
    if pad:
        rng = np.random.default_rng(99)
        o.add_facts("pad", [np.arange(pad, dtype=np.uint32) + 1000], rng.uniform(0.2, 0.9, pad).astype(np.float32))
    o.add_facts("edge", [src, dst], p)
    return o.run()


@pytest.mark.parametrize("pad", [70, 150])
@pytest.mark.parametrize("k", [1, 3])
def test_shift_invariance(oracle, synth, pad, k):
    src, dst, p = synth.er_graph(5, 14, 36, weights=True)
    base = run(oracle, src, dst, p, 0, k=k).read("path")
    wide = run(oracle, src, dst, p, pad, k=k).read("path")
    assert np.array_equal(base["cols"], wide["cols"])
    assert np.array_equal(base["cnt"], wide["cnt"])
    assert np.array_equal(base["p"], wide["p"])
    assert np.array_equal(base["prob"], wide["prob"])
    assert np.all(base["bits_wide"][:, :, 1:] == 0)  # 36 facts: one word
    for i in range(base["cols"].shape[0]):
        for j in range(int(base["cnt"][i])):
            assert as_int(wide["bits_wide"][i, j]) == as_int(base["bits_wide"][i, j]) << pad


def chain(n=100, seed=3):
    rng = np.random.default_rng(seed)
    src = np.arange(n, dtype=np.uint32)
    dst = src + 1
    q = rng.uniform(0.9, 0.999, n).astype(np.float32)
    # the bypass 0 -> n is fact n
    return np.append(src, 0).astype(np.uint32), np.append(dst, n).astype(np.uint32), np.append(q, np.float32(0.5))


def seq_prod(q):
    acc = np.float32(1.0)
    for x in q:
        acc = np.float32(acc * x)
    return acc


def test_chain_closed_form(oracle):
    n = 100
    src, dst, q = chain(n)
    r = run(oracle, src, dst, q).read("path")
    rows = {tuple(c): i for i, c in enumerate(r["cols"].tolist())}
    for a, b in [(0, 1), (0, 63), (0, 64), (3, 70), (10, 99), (60, 100), (1, 100)]:
        i = rows[(a, b)]
        assert r["cnt"][i] == 1
        want = sum(1 << f for f in range(a, b))  # edges a .. b-1
        assert as_int(r["bits_wide"][i, 0]) == want, (a, b)
        assert r["p"][i, 0] == seq_prod(q[a:b])
        assert r["prob"][i] == pytest.approx(np.prod(q[a:b].astype(np.float64)), rel=1e-12)
    # path(0, n): the bypass (fact n) and the whole chain (facts 0 .. n-1)
    i = rows[(0, n)]
    assert r["cnt"][i] == 2
    assert as_int(r["bits_wide"][i, 0]) == 1 << n and r["p"][i, 0] == np.float32(0.5)
    assert as_int(r["bits_wide"][i, 1]) == (1 << n) - 1 and r["p"][i, 1] == seq_prod(q[:n])
    c = np.prod(q[:n].astype(np.float64))
    assert r["prob"][i] == pytest.approx(0.5 + c - 0.5 * c, rel=1e-12)


def test_chain_gradient(oracle):
    n = 100
    src, dst, q = chain(n)
    o = run(oracle, src, dst, q, sr="diff_topk")
    r = o.read("path")
    g = np.zeros(r["cols"].shape[0])
    i = [t for t, c in enumerate(r["cols"].tolist()) if c == [0, n]][0]
    g[i] = 1.0
    o.backward("path", g)
    grad = o.grad("edge", n + 1)
    qd = q.astype(np.float64)
    c = np.prod(qd[:n])
    # P = a + c - a c with a the bypass: dP/da = 1 - c, dP/dq_j = (1 - a) c / q_j
    assert grad[n] == pytest.approx(1 - c, rel=1e-10)
    np.testing.assert_allclose(grad[:n], (1 - qd[n]) * c / qd[:n], rtol=1e-10)


def test_more_than_256_facts_refused(oracle):
    o = oracle.Oracle(TC, "topk", k=3)
    with pytest.raises(Exception):
        o.add_facts("pad", [np.arange(257, dtype=np.uint32)], np.full(257, 0.5, np.float32))
