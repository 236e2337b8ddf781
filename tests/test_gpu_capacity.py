"""Capacity paths on the GPU, forced at small sizes: joins whose outputs pass
the per-launch limit run in chunks of probe rows (max_join_outputs), and
buffers grown to exactly the size asked are regrown many times
(exact_growth).  Results must equal the CPU oracle's."""
import json

import numpy as np
import pytest

from gpu_util import (DEDUP, assert_tags_close, check_closure, engine, oracle_run, same_rows, tc_closure,
                      tune_key)

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dedup", [1, 2])
@pytest.mark.parametrize("sr", ["bool", "maxmin", "minplus", "addmult"])
def test_tc_chunked_joins(oracle, synth, sr, dedup, tmp_path):
    """Recent-driven joins (so every round goes through the general join
    driver) cut into chunks of at most 5000 outputs."""
    from paper_2503_21937_amd import dlfix
    n, m = 900, 3600
    src, dst, p = synth.er_graph(6, n, m, weights=True)
    e = dlfix.Engine(synth.TC_PROGRAM, sr, max_join_outputs=5000, exact_growth=True)
    e.add_facts("edge", [src, dst], None if sr == "bool" else p)
    key = tune_key(e)
    cache = tmp_path / "force.jsonl"
    cache.write_text(json.dumps({"key": key, "dedup": dedup, "orient": 1, "items": 2, "rows": 1, "ms": 1.0}) + "\n")
    e.autotune(1, str(cache))
    check_closure(e.read("path"), tc_closure(oracle, n, src, dst, p, sr), sr, f"chunked dedup={dedup}")
    assert e.stats()["candidates"] > 5000 * 10  # many chunks did run


@pytest.mark.parametrize("dedup", DEDUP)
def test_points_to_chunked(oracle, synth, dedup):
    """Three-atom rules: chunks of the first join each go through the second."""
    rels = synth.andersen(2, v=600, n_addr=300, n_assign=1800, n_load=240, n_store=240)
    facts = {name: ([a, b], None, None) for name, (a, b) in rels.items()}
    g = engine(synth.ANDERSEN_PROGRAM, "bool", facts, dedup=dedup, max_join_outputs=2000, exact_growth=True)
    o = oracle_run(oracle, synth.ANDERSEN_PROGRAM, "bool", facts)
    assert np.array_equal(g.read("pt")["cols"], o.read("pt")["cols"])
    assert g.stats()["max_rounds"] == o.rounds()


@pytest.mark.parametrize("dedup", DEDUP)
def test_grids_chunked_with_lineage(oracle, synth, dedup):
    """Differentiable add-mult with recorded lineage through chunked joins:
    tags and input gradients equal the oracle's."""
    g = synth.grid_batch(8, samples=10, kmin=3, kmax=8)
    facts = {"edge": ([g["src"], g["dst"]], g["p"], g["sample"])}
    e = engine(synth.TC_PROGRAM, "diff_addmult", facts, batched=True, dedup=dedup, lineage="store",
               max_join_outputs=1500, exact_growth=True)
    o = oracle_run(oracle, synth.TC_PROGRAM, "diff_addmult", facts, batched=True)
    gr, orr = e.read("path"), o.read("path")
    same_rows(gr, orr, batched=True)
    assert_tags_close(gr["tags"], orr["value"])
    gout = synth.normal_grads(3, orr["cols"].shape[0])
    e.backward("path", gout)
    o.backward("path", gout.astype(np.float64))
    n = g["src"].size
    np.testing.assert_allclose(e.grad("edge", n), o.grad("edge", n), rtol=1e-4, atol=1e-6)


def test_one_row_beyond_the_limit(synth):
    """A probe row whose matches alone pass the limit cannot be chunked."""
    from paper_2503_21937_amd import dlfix
    src = np.zeros(300, np.uint32)  # node 0 has 300 successors
    dst = np.arange(1, 301, dtype=np.uint32)
    prog = ".input edge/2\nsib(x, y) :- edge(p, x), edge(p, y).\n"
    e = dlfix.Engine(prog, "bool", dedup="sort", max_join_outputs=100)
    e.add_facts("edge", [src, dst])
    with pytest.raises(dlfix.DLError) as ex:
        e.run()
    assert ex.value.status == 6  # DL_ERR_CAPACITY
