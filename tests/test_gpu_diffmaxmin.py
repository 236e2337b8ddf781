"""GPU parity of the differentiable max-min semiring (tags: the probability
of one input fact and that fact's number) against the CPU oracle: values
and fact numbers bit-exact (both sides only ever pick among input
probabilities, with the same tie rule), input gradients equal up to the
order of float32 additions: a fact's gradient is the sum of the m output
gradients routed to it, added in any order in binary32, so it lies within
m * 2^-24 * sum|g| of the exact sum (the bound of recursive summation)."""
import numpy as np
import pytest

from gpu_util import engine, oracle_run, same_rows

pytestmark = pytest.mark.gpu


NONLINEAR = ".input edge/2\npath(x, y) :- edge(x, y).\npath(x, z) :- path(x, y), path(y, z).\n"


def check(g, o, rel, batched=False):
    gr, orr = g.read(rel), o.read(rel)
    same_rows(gr, orr, batched)
    assert np.array_equal(gr["tags"].astype(np.float64), orr["value"]), "values differ"
    assert np.array_equal(gr["fid"], o.fid(rel)), "fact numbers differ"
    return gr


def summation_bound(fid, g, nfacts):
    """Per fact: m * 2^-24 * sum |g| over the m outputs routed to it."""
    m = np.bincount(fid, minlength=nfacts).astype(np.float64)
    a = np.bincount(fid, weights=np.abs(g.astype(np.float64)), minlength=nfacts)
    return m * 2.0**-24 * a


def assert_grads(g, o, inputs, bound):
    off = 0
    for name, m in inputs.items():  # fact numbers run over the relations in add order
        got = g.grad(name, m).astype(np.float64)
        want = o.grad(name, m)
        b = bound[off:off + m]
        bad = np.abs(got - want) > b
        assert not bad.any(), (name, np.flatnonzero(bad)[:5], got[bad][:5], want[bad][:5], b[bad][:5])
        off += m


def check_grads(g, o, rel, inputs, seed):
    n = g.size(rel)
    gout = np.random.default_rng(seed).standard_normal(n).astype(np.float32)
    g.backward(rel, gout)
    o.backward(rel, gout.astype(np.float64))
    assert_grads(g, o, inputs, summation_bound(o.fid(rel).astype(np.int64), gout, sum(inputs.values())))


@pytest.mark.parametrize("program", ["linear", "nonlinear"])
@pytest.mark.parametrize("seed", [1, 2])
def test_tc(oracle, synth, program, seed):
    src, dst, p = synth.er_graph(seed, 400, 1600, weights=True)
    prog = synth.TC_PROGRAM if program == "linear" else NONLINEAR
    facts = {"edge": ([src, dst], p, None)}
    g = engine(prog, "diff_maxmin", facts)
    o = oracle_run(oracle, prog, "diff_maxmin", facts)
    check(g, o, "path")
    assert g.stats()["max_rounds"] == o.rounds()
    check_grads(g, o, "path", {"edge": src.size}, seed)


def test_ties_and_duplicates(oracle):
    """Every probability drawn from 4 values (many equal widest paths) and
    every edge given twice with different probabilities: the tie rule picks
    the smallest fact number on both sides."""
    rng = np.random.default_rng(7)
    n, m = 120, 500
    src = rng.integers(0, n, m).astype(np.uint32)
    dst = rng.integers(0, n, m).astype(np.uint32)
    src, dst = np.concatenate([src, src]), np.concatenate([dst, dst])
    p = np.array([0.25, 0.5, 0.75, 1.0], np.float32)[rng.integers(0, 4, 2 * m)]
    facts = {"edge": ([src, dst], p, None)}
    g = engine(NONLINEAR, "diff_maxmin", facts)
    o = oracle_run(oracle, NONLINEAR, "diff_maxmin", facts)
    check(g, o, "path")
    check_grads(g, o, "path", {"edge": 2 * m}, 3)


def test_batched_grids(oracle, synth):
    g_ = synth.grid_batch(5, samples=12, kmin=3, kmax=9)
    facts = {"edge": ([g_["src"], g_["dst"]], g_["p"], g_["sample"])}
    g = engine(synth.TC_PROGRAM, "diff_maxmin", facts, batched=True)
    o = oracle_run(oracle, synth.TC_PROGRAM, "diff_maxmin", facts, batched=True)
    check(g, o, "path", batched=True)
    check_grads(g, o, "path", {"edge": g_["src"].size}, 4)


def test_points_to_over_four_relations(oracle, synth):
    """Fact numbers run over all input relations in add order."""
    rels = synth.andersen(3, v=300, n_addr=150, n_assign=900, n_load=120, n_store=120)
    rng = np.random.default_rng(5)
    facts = {name: ([a, b], rng.uniform(0.05, 1.0, a.size).astype(np.float32), None)
             for name, (a, b) in rels.items()}
    g = engine(synth.ANDERSEN_PROGRAM, "diff_maxmin", facts)
    o = oracle_run(oracle, synth.ANDERSEN_PROGRAM, "diff_maxmin", facts)
    check(g, o, "pt")
    check_grads(g, o, "pt", {name: a.size for name, (a, _) in rels.items()}, 6)


def test_rows_seeded_backward(oracle, synth):
    """Gradients seeded on looked-up rows (absent tuples give -1 and are
    skipped) equal a full backward whose other rows carry zero."""
    src, dst, p = synth.er_graph(9, 200, 700, weights=True)
    facts = {"edge": ([src, dst], p, None)}
    g = engine(synth.TC_PROGRAM, "diff_maxmin", facts)
    o = oracle_run(oracle, synth.TC_PROGRAM, "diff_maxmin", facts)
    rng = np.random.default_rng(2)
    qx = rng.integers(0, 200, 300).astype(np.uint32)
    qz = rng.integers(0, 200, 300).astype(np.uint32)
    rows, tags = g.lookup("path", [qx, qz])
    gq = rng.standard_normal(300).astype(np.float32)
    g.backward_rows("path", rows, gq)
    full = np.zeros(g.size("path"), np.float64)
    np.add.at(full, rows[rows >= 0], gq[rows >= 0].astype(np.float64))
    o.backward("path", full)
    hit = rows >= 0
    fid = o.fid("path").astype(np.int64)[rows[hit]]
    assert_grads(g, o, {"edge": src.size}, summation_bound(fid, gq[hit], src.size))
    vals = o.read("path")["value"]
    assert np.array_equal(tags[rows >= 0].astype(np.float64), vals[rows[rows >= 0]])
    assert np.all(tags[rows < 0] == 0)


def test_dense_dedup_is_refused(synth):
    from paper_2503_21937_amd import dlfix
    src, dst, p = synth.er_graph(1, 50, 100, weights=True)
    e = dlfix.Engine(synth.TC_PROGRAM, "diff_maxmin", dedup="dense")
    e.add_facts("edge", [src, dst], p)
    with pytest.raises(dlfix.DLError) as ex:
        e.run()
    assert ex.value.status == 3  # DL_ERR_UNSUPPORTED
