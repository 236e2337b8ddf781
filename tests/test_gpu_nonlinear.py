"""GPU parity of rules with several atoms of their own stratum (non-linear and
mutual recursion).  Under frozen add-mult tags these use the stable / recent /
full delta split (Appendix A), so every discovery-round derivation is summed
exactly once; the converging semirings use the plain recent / full split."""
import numpy as np
import pytest

from gpu_util import DEDUP, assert_tags_close, engine, oracle_run, same_rows

pytestmark = pytest.mark.gpu

NONLINEAR = ".input edge/2\npath(x, y) :- edge(x, y).\npath(x, z) :- path(x, y), path(y, z).\n"
NONLINEAR3 = (".input edge/2\npath(x, y) :- edge(x, y).\n"
              "path(x, w) :- path(x, y), path(y, z), path(z, w).\n")
MUTUAL = (".input edge/2\na(x, y) :- edge(x, y).\nb(x, z) :- a(x, y), edge(y, z).\n"
          "a(x, z) :- b(x, y), a(y, z).\n")
SEMIRINGS = ["bool", "maxmin", "minplus", "addmult", "diff_addmult"]


def small_probs(rng, n):
    # small probabilities keep the frozen sums below the clamp at 1
    return rng.uniform(0.02, 0.2, n).astype(np.float32)


def check(oracle, program, sr, facts, rels, dedup):
    g = engine(program, sr, facts, dedup=dedup)
    o = oracle_run(oracle, program, sr, facts)
    for rel in rels:
        gr, orr = g.read(rel), o.read(rel)
        same_rows(gr, orr)
        if sr != "bool":
            assert_tags_close(gr["tags"], orr["value"], what=f"{sr} {rel}")
    if sr != "minplus":
        assert g.stats()["max_rounds"] == o.rounds()
    return g, o


@pytest.mark.parametrize("dedup", DEDUP)
@pytest.mark.parametrize("sr", SEMIRINGS)
def test_nonlinear_chain(oracle, sr, dedup):
    n = 40
    rng = np.random.default_rng(1)
    src = np.arange(n - 1, dtype=np.uint32)
    check(oracle, NONLINEAR, sr, {"edge": ([src, src + 1], small_probs(rng, n - 1), None)}, ["path"], dedup)


@pytest.mark.parametrize("dedup", DEDUP)
@pytest.mark.parametrize("seed", [1, 2])
@pytest.mark.parametrize("sr", SEMIRINGS)
def test_nonlinear_er(oracle, synth, sr, seed, dedup):
    src, dst, _ = synth.er_graph(seed, 96, 200, weights=True)
    p = small_probs(np.random.default_rng(seed), src.size)
    check(oracle, NONLINEAR, sr, {"edge": ([src, dst], p, None)}, ["path"], dedup)


@pytest.mark.parametrize("dedup", DEDUP)
@pytest.mark.parametrize("sr", ["bool", "maxmin", "addmult"])
def test_three_recursive_atoms(oracle, synth, sr, dedup):
    src, dst, _ = synth.er_graph(4, 80, 150, weights=True)
    p = small_probs(np.random.default_rng(4), src.size)
    check(oracle, NONLINEAR3, sr, {"edge": ([src, dst], p, None)}, ["path"], dedup)


@pytest.mark.parametrize("dedup", DEDUP)
@pytest.mark.parametrize("sr", SEMIRINGS)
def test_mutual_recursion(oracle, synth, sr, dedup):
    src, dst, _ = synth.er_graph(6, 120, 300, weights=True)
    p = small_probs(np.random.default_rng(6), src.size)
    check(oracle, MUTUAL, sr, {"edge": ([src, dst], p, None)}, ["a", "b"], dedup)


@pytest.mark.parametrize("dedup", DEDUP)
def test_nonlinear_gradients(oracle, synth, dedup):
    src, dst, _ = synth.er_graph(3, 64, 140, weights=True)
    p = small_probs(np.random.default_rng(3), src.size)
    facts = {"edge": ([src, dst], p, None)}
    g, o = check(oracle, NONLINEAR, "diff_addmult", facts, ["path"], dedup)
    n = o.size("path")
    gout = np.random.default_rng(9).normal(size=n)
    g.backward("path", gout.astype(np.float32))
    o.backward("path", gout)
    np.testing.assert_allclose(g.grad("edge", src.size), o.grad("edge", src.size), rtol=1e-4, atol=1e-6)


# Same Generation without its inequality (arithmetic selections are not
# supported): a recursive atom between two static atoms, planned as two binary
# joins through an intermediate relation (differentiable add-mult records
# derivations of at most two body atoms, so it is not among the semirings).
SAME_GEN = (".input edge/2\nsg(x, y) :- edge(p, x), edge(p, y).\n"
            "sg(x, y) :- edge(a, x), sg(a, b), edge(b, y).\n")


@pytest.mark.parametrize("dedup", DEDUP)
@pytest.mark.parametrize("sr", ["bool", "maxmin", "minplus", "addmult"])
def test_same_generation(oracle, synth, sr, dedup):
    src, dst, _ = synth.er_graph(8, 60, 110, weights=True)
    p = small_probs(np.random.default_rng(8), src.size)
    check(oracle, SAME_GEN, sr, {"edge": ([src, dst], p, None)}, ["sg"], dedup)
