"""Same Generation (a non-linear recursion with a selection) on the
transitive-closure graphs: GPU against the CPU oracle on the small graph
under every tag semiring, and at the benchmark graph's full size against a
closed form of the tuple set computed here with sparse boolean matrices.

    sg(x, y) :- edge(p, x), edge(p, y), x != y.
    sg(x, y) :- edge(a, x), sg(a, b), edge(b, y).

As sets of pairs (S, E boolean n x n): S is the least solution of
S = (E^T E minus its diagonal) | E^T S E.
"""
import numpy as np
import pytest

from gpu_util import DEDUP, assert_tags_close, engine, oracle_run, same_rows
from test_oracle_eval import SG

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dedup", DEDUP)
@pytest.mark.parametrize("sr", ["bool", "maxmin", "minplus", "addmult"])
def test_sg_er256(oracle, synth, sr, dedup):
    src, dst, p = synth.er_graph(1, 256, 1024, weights=True)
    facts = {"edge": ([src, dst], None if sr == "bool" else p, None)}
    g = engine(SG, sr, facts, dedup=dedup)
    o = oracle_run(oracle, SG, sr, facts)
    gr, orr = g.read("sg"), o.read("sg")
    same_rows(gr, orr)
    if sr == "maxmin":
        assert np.array_equal(gr["tags"].astype(np.float64), orr["value"])
    elif sr != "bool":
        assert_tags_close(gr["tags"], orr["value"], what=sr)
    if sr != "minplus":
        assert g.stats()["max_rounds"] == o.rounds()


def sg_closed_form(n, src, dst):
    import scipy.sparse as sp
    E = sp.csr_matrix((np.ones(src.size, np.float32), (src, dst)), shape=(n, n))
    base = (E.T @ E).toarray() > 0
    np.fill_diagonal(base, False)
    S = base.copy()
    while True:
        # E^T S E as (E^T (S E)): sparse x dense products
        SE = (E.T @ S.astype(np.float32).T).T  # S @ E
        nxt = base | ((E.T @ SE) > 0)
        if np.array_equal(nxt, S):
            return S
        S = nxt


@pytest.mark.parametrize("dedup", ["dense"])
def test_sg_er5000_set(synth, dedup):
    n, m = 5000, 20000
    src, dst, p = synth.er_graph(1, n, m, weights=True)
    want = sg_closed_form(n, src, dst)
    for sr in ("bool", "maxmin"):
        g = engine(SG, sr, {"edge": ([src, dst], None if sr == "bool" else p, None)}, dedup=dedup)
        cols = g.read("sg")["cols"]
        assert cols.shape[0] == int(want.sum()), sr
        got = np.zeros((n, n), bool)
        got[cols[:, 0], cols[:, 1]] = True
        assert np.array_equal(got, want), sr
