"""Edge cases of the newer paths on the GPU, against the CPU oracle where
there is a result: empty inputs and empty rounds for hash indexes, hash-set
deduplication, fused rounds and the differentiable max-min semiring, the
one-word / four-word boundary of top-k proof sets (64 and 65 probabilistic
facts in a sample), and the round log of an engine without facts."""
import json

import numpy as np
import pytest

from gpu_util import assert_tags_close, engine, oracle_run, same_rows, tune_key

pytestmark = pytest.mark.gpu

TC = ".input edge/2\npath(x, y) :- edge(x, y).\npath(x, z) :- edge(x, y), path(y, z).\n"


# differentiable max-min always takes the sort-based pipeline
@pytest.mark.parametrize("sr,dedup", [(sr, d) for sr in ("bool", "maxmin") for d in ("sort", "dense", "hash")] +
                         [("diff_maxmin", "sort"), ("diff_maxmin", "hash")])
def test_no_facts(sr, dedup):
    from paper_2503_21937_amd import dlfix
    e = dlfix.Engine(TC, sr, dedup=dedup)
    e.run()
    assert e.size("path") == 0
    r = e.read("path")
    assert r["cols"].shape == (0, 2)
    log = e.round_log()
    assert log["kind"].size >= 1 and int(log["new"].sum()) == 0
    if sr == "diff_maxmin":
        e.backward("path", np.zeros(0, np.float32))


@pytest.mark.parametrize("dedup", ["sort", "dense", "hash"])
def test_no_second_round(oracle, dedup):
    """Edges without any 2-path: round 2 finds nothing (fused rounds end at
    their first launch)."""
    src = np.arange(0, 200, 2, dtype=np.uint32)
    dst = src + 1
    facts = {"edge": ([src, dst], np.full(src.size, 0.5, np.float32), None)}
    g = engine(TC, "maxmin", facts, dedup=dedup)
    o = oracle_run(oracle, TC, "maxmin", facts)
    same_rows(g.read("path"), o.read("path"))
    assert g.stats()["max_rounds"] == o.rounds() == 2


def test_hash_index_with_empty_side(synth, tmp_path):
    """A join whose indexed side is empty under forced hash indexes."""
    from paper_2503_21937_amd import dlfix
    prog = ".input a/2\n.input b/2\nc(x, z) :- a(x, y), b(y, z).\n"
    e = dlfix.Engine(prog, "bool", dedup="sort")
    e.add_facts("a", [np.arange(10, dtype=np.uint32), np.arange(10, dtype=np.uint32)])
    key = tune_key(e)
    cache = tmp_path / "f.jsonl"
    cache.write_text(json.dumps({"key": key, "dedup": 1, "orient": 1, "items": 2, "rows": 1, "index": 1,
                                 "ms": 1.0}) + "\n")
    e.autotune(1, str(cache))
    assert e.stats()["index"] == 1 and e.size("c") == 0


@pytest.mark.parametrize("nfacts", [64, 65])
def test_topk_word_boundary(oracle, nfacts):
    """64 probabilistic facts in a sample keep one-word proof sets, 65 take
    four; both agree with the oracle."""
    rng = np.random.default_rng(nfacts)
    src = rng.integers(0, 20, nfacts).astype(np.uint32)
    dst = rng.integers(0, 20, nfacts).astype(np.uint32)
    p = rng.uniform(0.3, 0.95, nfacts).astype(np.float32)
    facts = {"edge": ([src, dst], p, None)}
    g = engine(TC, "diff_topk", facts, k=3)
    o = oracle_run(oracle, TC, "diff_topk", facts, k=3)
    gr, orr = g.read("path"), o.read("path")
    same_rows(gr, orr)
    words = g.stats()["topk_words"]
    assert words == (1 if nfacts <= 64 else 4)
    want = orr["bits_wide"][:, :3, 0] if words == 1 else orr["bits_wide"][:, :3, :]
    assert np.array_equal(gr["bits"], want)
    assert np.array_equal(gr["p"], orr["p"])
    assert_tags_close(gr["tags"], orr["prob"])
    gout = np.random.default_rng(1).standard_normal(orr["cols"].shape[0]).astype(np.float32)
    g.backward("path", gout)
    o.backward("path", gout.astype(np.float64))
    np.testing.assert_allclose(g.grad("edge", nfacts), o.grad("edge", nfacts), rtol=1e-4, atol=1e-6)


def test_clear_facts_resets_fact_numbers(oracle, synth):
    """Differentiable max-min numbers facts from 0 again after dl_clear_facts."""
    from paper_2503_21937_amd import dlfix
    src, dst, p = synth.er_graph(2, 60, 150, weights=True)
    e = dlfix.Engine(TC, "diff_maxmin")
    e.add_facts("edge", [src[:50], dst[:50]], p[:50])
    e.run()
    e.clear_facts()
    e.add_facts("edge", [src, dst], p)
    e.run()
    o = oracle_run(oracle, TC, "diff_maxmin", {"edge": ([src, dst], p, None)})
    assert np.array_equal(e.read("path")["fid"], o.fid("path"))
