"""Parity at the benchmark's full size: probabilistic reachability on the
seeded directed G(5000, 20000) graph (seed 1), under add-mult, max-min and
min-plus, in the execution configuration the autotuner picks for the bench
and in every candidate configuration it chooses among.

The oracle side is the column solver (every target column z of the
transitive closure evolves on its own, round for round, as in the full naive
Jacobi evaluation), run for all 5000 columns on a thread pool, so the whole
relation is compared element by element: tuple sets exact, max-min tags
bit-exact, add-mult and min-plus tags within 1e-5 relative, and the round
count of the fixpoint (the largest round count over the columns; min-plus
excluded: binary32 sums against the binary64 oracle may move a tie by one
round).
"""
import concurrent.futures as cf
import json

import numpy as np
import pytest

from gpu_util import assert_tags_close, tune_key

pytestmark = pytest.mark.gpu

N, M, SEED = 5000, 20000, 1
SEMIRINGS = ["addmult", "maxmin", "minplus"]
# the autotuner's candidates: (dedup, orient, items, rows)
CONFIGS = [(d, o, it, 1) for d in (1, 2) for o in (1, 2) for it in (1, 2, 4, 8)]
CONFIGS += [(2, 2, it, 0) for it in (1, 2, 4, 8)]


@pytest.fixture(scope="module")
def graph(synth):
    return synth.er_graph(SEED, N, M, weights=True)


@pytest.fixture(scope="module")
def columns(oracle, graph):
    """sr -> (present[x, z], tag[x, z], rounds) from the oracle, all columns."""
    src, dst, p = graph
    out = {}
    for sr in SEMIRINGS:
        pres = np.zeros((N, N), bool)
        tag = np.zeros((N, N), np.float64)
        rounds = np.zeros(N, np.int64)

        def col(z):
            c = oracle.tc_column(N, src, dst, p, sr, z)
            pres[:, z] = c["present"]
            tag[:, z] = c["tag"]
            rounds[z] = c["rounds"]

        with cf.ThreadPoolExecutor(16) as ex:  # ctypes calls release the GIL
            list(ex.map(col, range(N)))
        out[sr] = (pres, tag, int(rounds.max()))
    return out


def check(e, sr, want, what):
    pres, tag, rounds = want
    r = e.read("path")
    cols = r["cols"]
    got = np.zeros((N, N), bool)
    got[cols[:, 0], cols[:, 1]] = True
    assert cols.shape[0] == int(pres.sum()), what
    assert np.array_equal(got, pres), what
    ref = tag[cols[:, 0], cols[:, 1]]
    if sr == "maxmin":
        assert np.array_equal(r["tags"].astype(np.float64), ref), what
    else:
        assert_tags_close(r["tags"], ref, what=what)
    if sr != "minplus":
        assert e.stats()["max_rounds"] == rounds, what


@pytest.mark.parametrize("sr", SEMIRINGS)
def test_autotuned_configuration(synth, graph, columns, sr, tmp_path):
    from paper_2503_21937_amd import dlfix
    src, dst, p = graph
    e = dlfix.Engine(synth.TC_PROGRAM, sr)
    e.add_facts("edge", [src, dst], p)
    cfg = e.autotune(1, str(tmp_path / "tune.jsonl"))
    check(e, sr, columns[sr], f"{sr} autotuned {cfg}")
    e.run()  # a second run on the same engine (buffers reused)
    check(e, sr, columns[sr], f"{sr} autotuned rerun")


@pytest.mark.parametrize("sr", SEMIRINGS)
def test_every_candidate_configuration(synth, graph, columns, sr, tmp_path):
    from paper_2503_21937_amd import dlfix
    src, dst, p = graph
    e = dlfix.Engine(synth.TC_PROGRAM, sr)
    e.add_facts("edge", [src, dst], p)
    key = tune_key(e)
    for dedup, orient, items, rows in CONFIGS:
        cache = tmp_path / f"force_{dedup}_{orient}_{items}_{rows}.jsonl"
        cache.write_text(json.dumps({"key": key, "dedup": dedup, "orient": orient, "items": items,
                                     "rows": rows, "ms": 1.0}) + "\n")
        cfg = e.autotune(1, str(cache))
        assert (cfg["dedup"], cfg["orient"], cfg["items"], cfg["rows"]) == (dedup, orient, items, rows)
        check(e, sr, columns[sr], f"{sr} config {(dedup, orient, items, rows)}")
