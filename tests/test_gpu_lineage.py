"""Reverse mode without recorded lineage: dl_backward recomputes every round's
discovery derivations from the relations as they stood (rebuilt from the
discovery ids).  Gradients must agree with the recorded-lineage sweep and the
CPU oracle."""
import numpy as np
import pytest

from gpu_util import DEDUP, assert_tags_close, engine, oracle_run, same_rows

pytestmark = pytest.mark.gpu

NONLINEAR = ".input edge/2\npath(x, y) :- edge(x, y).\npath(x, z) :- path(x, y), path(y, z).\n"
MUTUAL = (".input edge/2\na(x, y) :- edge(x, y).\nb(x, z) :- a(x, y), edge(y, z).\n"
          "a(x, z) :- b(x, y), a(y, z).\n")


def grads(e, rel, gout, n_in):
    e.zero_grad()
    e.backward(rel, gout.astype(np.float32))
    return e.grad("edge", n_in)


@pytest.mark.parametrize("dedup", DEDUP)
@pytest.mark.parametrize("mode", ["recompute", "budget"])
def test_grid_batch_recompute_vs_oracle(oracle, synth, dedup, mode):
    g = synth.grid_batch(4, samples=10, kmin=2, kmax=7)
    facts = {"edge": ([g["src"], g["dst"]], g["p"], g["sample"])}
    kw = dict(lineage="recompute") if mode == "recompute" else dict(lineage="auto", lineage_budget=2400)
    ge = engine(synth.TC_PROGRAM, "diff_addmult", facts, batched=True, dedup=dedup, **kw)
    st = ge.stats()
    assert st["lineage_mode"] == 2
    oe = oracle_run(oracle, synth.TC_PROGRAM, "diff_addmult", facts, batched=True)
    gr, orr = ge.read("path"), oe.read("path")
    same_rows(gr, orr, batched=True)
    assert_tags_close(gr["tags"], orr["value"])
    gout = np.random.default_rng(2).normal(size=orr["cols"].shape[0])
    gg = grads(ge, "path", gout, g["src"].size)
    oe.backward("path", gout)
    np.testing.assert_allclose(gg, oe.grad("edge", g["src"].size), rtol=1e-4, atol=1e-6)
    # the recorded sweep gives the same gradients
    se = engine(synth.TC_PROGRAM, "diff_addmult", facts, batched=True, dedup=dedup, lineage="store")
    assert se.stats()["lineage_mode"] == 1
    # (float atomics: the sums may be taken in another order)
    ref = grads(se, "path", gout, g["src"].size)
    np.testing.assert_allclose(gg, ref, rtol=1e-5, atol=1e-6 * np.abs(ref).max())


@pytest.mark.parametrize("dedup", DEDUP)
@pytest.mark.parametrize("program,rel", [(NONLINEAR, "path"), (MUTUAL, "a")])
def test_recursive_programs_recompute(oracle, synth, dedup, program, rel):
    src, dst, _ = synth.er_graph(8, 72, 160, weights=True)
    p = np.random.default_rng(8).uniform(0.02, 0.2, src.size).astype(np.float32)
    facts = {"edge": ([src, dst], p, None)}
    ge = engine(program, "diff_addmult", facts, dedup=dedup, lineage="recompute")
    oe = oracle_run(oracle, program, "diff_addmult", facts)
    gr, orr = ge.read(rel), oe.read(rel)
    same_rows(gr, orr)
    assert_tags_close(gr["tags"], orr["value"])
    gout = np.random.default_rng(3).normal(size=orr["cols"].shape[0])
    gg = grads(ge, rel, gout, src.size)
    oe.backward(rel, gout)
    np.testing.assert_allclose(gg, oe.grad("edge", src.size), rtol=1e-4, atol=1e-6)


def test_auto_records_when_it_fits(synth):
    g = synth.grid_batch(6, samples=4, kmin=3, kmax=5)
    facts = {"edge": ([g["src"], g["dst"]], g["p"], g["sample"])}
    e = engine(synth.TC_PROGRAM, "diff_addmult", facts, batched=True)
    st = e.stats()
    assert st["lineage_mode"] == 1 and st["lineage"] > 0
    assert engine(synth.TC_PROGRAM, "addmult", facts, batched=True).stats()["lineage_mode"] == 0
