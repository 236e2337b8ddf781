"""GPU parity of the fused rounds (one launch per round over a window-layout
recent relation) against the CPU oracle and against the same engine with
fused rounds switched off: batched samples (the general, multi-sample form
of the kernel), a three-column head, and the window / scatter choices
forced both ways."""
import json

import numpy as np
import pytest

from gpu_util import assert_tags_close, engine, oracle_run, same_rows, tune_key

pytestmark = pytest.mark.gpu


def check(g, o, rel, sr, batched=False):
    gr, orr = g.read(rel), o.read(rel)
    same_rows(gr, orr, batched)
    if sr == "maxmin":
        assert np.array_equal(gr["tags"].astype(np.float64), orr["value"])
    elif sr != "bool":
        assert_tags_close(gr["tags"], orr["value"], what=sr)


@pytest.mark.parametrize("sr", ["bool", "maxmin", "minplus", "addmult"])
def test_batched_samples(oracle, synth, sr):
    """Grids of several sizes in one engine: per-sample windows and groups."""
    g = synth.grid_batch(9, samples=24, kmin=3, kmax=12)
    facts = {"edge": ([g["src"], g["dst"]], None if sr == "bool" else g["p"], g["sample"])}
    o = oracle_run(oracle, synth.TC_PROGRAM, sr, facts, batched=True)
    for fused in (True, False):
        e = engine(synth.TC_PROGRAM, sr, facts, batched=True, dedup="dense", fused=fused)
        check(e, o, "path", sr, batched=True)
        if sr != "minplus":
            assert e.stats()["max_rounds"] == o.rounds()


THREE = """
.input e/2
.input f/3
r(x, z, w) :- f(x, z, w).
r(x, z, w) :- e(x, y), r(y, z, w).
"""


@pytest.mark.parametrize("sr", ["bool", "maxmin", "addmult"])
def test_three_column_head(oracle, synth, sr):
    rng = np.random.default_rng(3)
    src, dst, p = synth.er_graph(2, 60, 150, weights=True)
    n = 80
    f = [rng.integers(0, 60, n).astype(np.uint32), rng.integers(0, 60, n).astype(np.uint32),
         rng.integers(0, 60, n).astype(np.uint32)]
    fp = synth.unit_prob(rng, n)
    facts = {"e": ([src, dst], None if sr == "bool" else p, None), "f": (f, None if sr == "bool" else fp, None)}
    o = oracle_run(oracle, THREE, sr, facts)
    for fused in (True, False):
        e = engine(THREE, sr, facts, dedup="dense", fused=fused)
        check(e, o, "r", sr)


@pytest.mark.parametrize("rows", [0, 2])
@pytest.mark.parametrize("sr", ["maxmin", "addmult", "bool"])
def test_window_and_scatter_forced(oracle, synth, sr, rows, tmp_path):
    """Every group folded in LDS (rows = 2) or every group scattered with
    global atomics (rows = 0), forced through the autotuner's cache."""
    from gpu_util import tc_closure, check_closure
    from paper_2503_21937_amd import dlfix
    n, m = 1500, 6000
    src, dst, p = synth.er_graph(4, n, m, weights=True)
    e = dlfix.Engine(synth.TC_PROGRAM, sr)
    e.add_facts("edge", [src, dst], None if sr == "bool" else p)
    key = tune_key(e)
    cache = tmp_path / "force.jsonl"
    cache.write_text(json.dumps({"key": key, "dedup": 2, "orient": 2, "items": 2, "rows": rows, "ms": 1.0}) + "\n")
    e.autotune(1, str(cache))
    check_closure(e.read("path"), tc_closure(oracle, n, src, dst, p, sr), sr, f"rows={rows}")


@pytest.mark.parametrize("sr", ["maxmin", "addmult"])
def test_round_log(synth, sr):
    """One log entry per fused launch: the rounds after the first come in
    order until one finds nothing (later launches of that batch find nothing
    too), and their derivations add up to the fused part of the candidates."""
    from paper_2503_21937_amd import dlfix
    src, dst, p = synth.er_graph(5, 2000, 8000, weights=True)
    on = dlfix.Engine(synth.TC_PROGRAM, sr, dedup="dense")
    on.add_facts("edge", [src, dst], p)
    on.run()
    log = on.round_log()
    kinds = log["kind"]
    assert kinds[0] == 1 and np.all(kinds[1:] == 3)  # round 1, then fused launches
    new, der = log["new"][1:], log["derivations"][1:]
    assert int(log["derivations"][0]) == src.size  # round 1 derives one candidate per edge
    st = on.stats()
    first_empty = int(np.argmax(new == 0))
    assert new[first_empty] == 0 and np.all(new[first_empty:] == 0) and np.all(der[first_empty + 1:] == 0)
    assert first_empty + 1 == st["max_rounds"] - 1  # round 1 is not fused; its last round finds nothing
    off = dlfix.Engine(synth.TC_PROGRAM, sr, dedup="dense", fused=False)
    off.add_facts("edge", [src, dst], p)
    off.run()
    olog = off.round_log()
    assert olog["kind"][0] == 1 and set(olog["kind"][1:].tolist()) <= {2, 4}
    # the same rounds and new or changed tuples either way
    assert int(olog["new"].sum()) == int(log["new"].sum())
    assert olog["kind"].size == st["max_rounds"]  # one entry per round, the last finding nothing
    # the same derivations either way; round 1 (the base rule) derives one
    # candidate per edge
    assert st["candidates"] == off.stats()["candidates"]
    assert int(der.sum()) + src.size == st["candidates"]


@pytest.mark.parametrize("sr", ["maxmin", "addmult"])
def test_graphs_kept_across_runs(oracle, synth, sr):
    """The fused rounds' graphs stay in the engine from run to run while
    their launches' arguments are the same: new facts of the same shape
    reuse them (the graphs read the buffers' new contents), facts of another
    shape make new ones; every run agrees with the oracle."""
    from paper_2503_21937_amd import dlfix
    e = dlfix.Engine(synth.TC_PROGRAM, sr, dedup="dense")
    ref = {}
    for seed, n, m in [(11, 200, 800), (11, 200, 800), (12, 200, 800), (13, 260, 1000), (12, 200, 800)]:
        src, dst, p = synth.er_graph(seed, n, m, weights=True)
        e.clear_facts()
        e.add_facts("edge", [src, dst], p)
        e.run()
        if seed not in ref:
            ref[seed] = oracle_run(oracle, synth.TC_PROGRAM, sr, {"edge": ([src, dst], p, None)})
        o = ref[seed]
        check(e, o, "path", sr)
        assert e.stats()["max_rounds"] == o.rounds()
