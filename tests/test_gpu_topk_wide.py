"""GPU parity of top-k proofs over more than 64 probabilistic facts per
sample (four-word proof sets) against the CPU oracle: proof sets, proof
probabilities (the same binary32 products), the inclusion-exclusion
probability and its gradient, on instances whose proofs lie above fact 64
(unused facts numbered first), a 100-edge chain with a bypass, and batched
samples of mixed sizes."""
import numpy as np
import pytest

from gpu_util import assert_tags_close, engine, oracle_run, same_rows

pytestmark = pytest.mark.gpu

TC = """
.input pad/1
.input edge/2
path(x, y) :- edge(x, y).
path(x, z) :- path(x, y), edge(y, z).
"""


def check(g, o, rel, k, batched=False):
    gr, orr = g.read(rel), o.read(rel)
    same_rows(gr, orr, batched)
    assert g.stats()["topk_words"] == 4
    assert gr["bits"].shape[1:] == (k, 4)
    assert np.array_equal(gr["cnt"].astype(np.int32), orr["cnt"])
    assert np.array_equal(gr["bits"], orr["bits_wide"][:, :k, :]), rel
    assert np.array_equal(gr["p"][:, :k], orr["p"][:, :k]), rel
    assert_tags_close(gr["tags"], orr["prob"], what=rel)


def grads(g, o, rel, inputs, seed):
    n = o.size(rel)
    gout = np.random.default_rng(seed).standard_normal(n).astype(np.float32)
    g.backward(rel, gout)
    o.backward(rel, gout.astype(np.float64))
    for name, m in inputs.items():
        np.testing.assert_allclose(g.grad(name, m), o.grad(name, m), rtol=1e-4, atol=1e-6, err_msg=name)


@pytest.mark.parametrize("k", [1, 3])
@pytest.mark.parametrize("pad", [70, 150])
def test_proofs_above_fact_64(oracle, synth, pad, k):
    rng = np.random.default_rng(pad)
    src, dst, p = synth.er_graph(5, 14, 36, weights=True)
    facts = {"pad": ([np.arange(pad, dtype=np.uint32) + 1000], rng.uniform(0.2, 0.9, pad).astype(np.float32), None),
             "edge": ([src, dst], p, None)}
    g = engine(TC, "diff_topk", facts, k=k)
    o = oracle_run(oracle, TC, "diff_topk", facts, k=k)
    check(g, o, "path", k)
    grads(g, o, "path", {"pad": pad, "edge": src.size}, 1)


def test_chain_with_bypass(oracle):
    n = 100
    rng = np.random.default_rng(3)
    src = np.append(np.arange(n, dtype=np.uint32), 0).astype(np.uint32)
    dst = np.append(np.arange(1, n + 1, dtype=np.uint32), n).astype(np.uint32)
    q = np.append(rng.uniform(0.9, 0.999, n).astype(np.float32), np.float32(0.5))
    facts = {"edge": ([src, dst], q, None)}
    g = engine(TC, "diff_topk", facts, k=3)
    o = oracle_run(oracle, TC, "diff_topk", facts, k=3)
    check(g, o, "path", 3)
    grads(g, o, "path", {"edge": n + 1}, 2)
    # seeded on one looked-up row
    g.zero_grad()
    o.zero_grad()
    rows, _ = g.lookup("path", [np.array([0], np.uint32), np.array([n], np.uint32)])
    g.backward_rows("path", rows, np.array([1.0], np.float32))
    full = np.zeros(o.size("path"))
    full[rows[0]] = 1.0
    o.backward("path", full)
    np.testing.assert_allclose(g.grad("edge", n + 1), o.grad("edge", n + 1), rtol=1e-4, atol=1e-7)


def test_batched_mixed_sizes(oracle, synth):
    """Samples of 20 to 200 probabilistic facts in one engine."""
    rng = np.random.default_rng(8)
    s_all, a_all, b_all, p_all = [], [], [], []
    for s in range(6):
        m = int(rng.integers(20, 201))
        nodes = int(rng.integers(10, 40))
        a = rng.integers(0, nodes, m).astype(np.uint32)
        b = rng.integers(0, nodes, m).astype(np.uint32)
        s_all.append(np.full(m, s, np.uint32))
        a_all.append(a)
        b_all.append(b)
        p_all.append(rng.uniform(0.3, 0.95, m).astype(np.float32))
    facts = {"edge": ([np.concatenate(a_all), np.concatenate(b_all)], np.concatenate(p_all), np.concatenate(s_all))}
    g = engine(TC, "diff_topk", facts, k=3, batched=True)
    o = oracle_run(oracle, TC, "diff_topk", facts, k=3, batched=True)
    check(g, o, "path", 3, batched=True)
    assert g.stats()["max_rounds"] == o.rounds()
    grads(g, o, "path", {"edge": sum(x.size for x in a_all)}, 3)
