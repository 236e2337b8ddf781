"""GPU parity of expression evaluation (comparisons in rule bodies, constants
and repeated variables in atoms, arithmetic head terms, nullary heads)
against the CPU oracle, through both deduplication pipelines."""
import numpy as np
import pytest

from gpu_util import DEDUP, assert_tags_close, engine, oracle_run, same_rows
from test_oracle_eval import FILTERS, PATHFINDER, REACH, SG, WALK, random_tree

pytestmark = pytest.mark.gpu

SEMIRINGS = ["bool", "maxmin", "minplus", "addmult"]


def compare(g, o, rel, sr, batched=False, what=""):
    gr, orr = g.read(rel), o.read(rel)
    assert gr["cols"].shape == orr["cols"].shape, (what, rel)
    same_rows(gr, orr, batched)
    if sr == "maxmin":
        assert np.array_equal(gr["tags"].astype(np.float64), orr["value"]), (what, rel)
    elif sr in ("minplus", "addmult", "diff_addmult"):
        assert_tags_close(gr["tags"], orr["value"], what=f"{what} {rel}")


def both(oracle, program, sr, facts, dedup, **kw):
    g = engine(program, sr, facts, dedup=dedup, **kw)
    o = oracle_run(oracle, program, sr, facts, **kw)
    return g, o


@pytest.mark.parametrize("dedup", DEDUP)
@pytest.mark.parametrize("sr", SEMIRINGS)
def test_same_generation_tree(oracle, sr, dedup):
    parent, p = random_tree(2, 300)
    src = parent[1:].astype(np.uint32)
    dst = np.arange(1, 300, dtype=np.uint32)
    g, o = both(oracle, SG, sr, {"edge": ([src, dst], None if sr == "bool" else p[1:], None)}, dedup)
    compare(g, o, "sg", sr, what="tree")
    assert g.stats()["max_rounds"] == o.rounds()


@pytest.mark.parametrize("dedup", DEDUP)
@pytest.mark.parametrize("sr", SEMIRINGS)
def test_same_generation_er(oracle, synth, sr, dedup):
    """Same Generation with its x != y selection on a random graph (several
    tiles of joins, both delta plans of the non-linear rule)."""
    src, dst, p = synth.er_graph(3, 120, 200, weights=True)
    g, o = both(oracle, SG, sr, {"edge": ([src, dst], None if sr == "bool" else p, None)}, dedup)
    compare(g, o, "sg", sr, what="er")
    if sr != "minplus":
        assert g.stats()["max_rounds"] == o.rounds()


@pytest.mark.parametrize("dedup", DEDUP)
@pytest.mark.parametrize("sr", SEMIRINGS)
def test_walks_with_arithmetic_heads(oracle, synth, sr, dedup):
    src, dst, p = synth.er_graph(4, 200, 600, weights=True)
    p = (p * 0.3).astype(np.float32)
    g, o = both(oracle, WALK.format(L=5), sr, {"edge": ([src, dst], None if sr == "bool" else p, None)}, dedup)
    compare(g, o, "walk", sr)


@pytest.mark.parametrize("dedup", DEDUP)
@pytest.mark.parametrize("sr", ["bool", "maxmin"])
def test_constants_and_nullary(oracle, synth, sr, dedup):
    for seed in (5, 6):
        src, dst, p = synth.er_graph(seed, 150, 170, weights=True)
        g, o = both(oracle, REACH, sr, {"edge": ([src, dst], None if sr == "bool" else p, None)}, dedup)
        for rel in ("path", "from0", "cyclic"):
            compare(g, o, rel, sr, what=f"seed {seed}")


@pytest.mark.parametrize("dedup", DEDUP)
def test_filters_repeats_division(oracle, dedup):
    rng = np.random.default_rng(6)
    src = rng.integers(0, 40, 3000).astype(np.uint32)
    dst = rng.integers(0, 40, 3000).astype(np.uint32)
    g, o = both(oracle, FILTERS, "bool", {"edge": ([src, dst], None, None)}, dedup)
    for rel in ("loop", "even_big", "ratio", "dbl"):
        compare(g, o, rel, "bool", what=rel)


@pytest.mark.parametrize("dedup", DEDUP)
def test_every_row_filtered(oracle, dedup):
    """A condition no derivation meets: empty results, no failure."""
    src = np.arange(0, 50, dtype=np.uint32)
    dst = src + 1
    prog = ".input edge/2\nq(x, y) :- edge(x, y), x > y.\nr(x) :- q(x, y).\nz() :- edge(x, y), y == 0.\n"
    g, o = both(oracle, prog, "bool", {"edge": ([src, dst], None, None)}, dedup)
    for rel in ("q", "r", "z"):
        assert g.size(rel) == 0 == o.size(rel)


@pytest.mark.parametrize("dedup", DEDUP)
@pytest.mark.parametrize("sr", ["bool", "topk", "diff_addmult"])
def test_pathfinder_batched(oracle, synth, sr, dedup):
    """The motivating program on a batch of grids with per-sample endpoints
    (conditions and a nullary head on batched keys).  Add-mult rules hold
    two body atoms, so its endpoint query takes two steps."""
    if sr == "topk" and dedup == "dense":
        pytest.skip("top-k tags always take the sort-based pipeline")
    # top-k: at most 64 probabilistic facts per sample, so grids up to 4 x 4
    g = synth.grid_batch(7, samples=12, kmin=3, kmax=4 if sr == "topk" else 6)
    rng = np.random.default_rng(7)
    es, ev = [], []
    for s, k in enumerate(g["ks"]):
        ends = rng.choice(int(k) * int(k), 2, replace=False)
        es += [s, s]
        ev += list(ends)
    es = np.array(es, np.uint32)
    ev = np.array(ev, np.uint32)
    ep = np.full(es.size, 0.9, np.float32)
    prog = PATHFINDER
    if sr == "diff_addmult":
        prog = (".input edge/2\n.input is_endpoint/1\npath(x, y) :- edge(x, y).\n"
                "path(x, z) :- path(x, y), edge(y, z).\n"
                "from_end(x, y) :- is_endpoint(x), path(x, y), x != y.\n"
                "endpoints_connected() :- from_end(x, y), is_endpoint(y).\n")
    facts = {"edge": ([g["src"], g["dst"]], g["p"], g["sample"]), "is_endpoint": ([ev], ep, es)}
    ge = engine(prog, sr, facts, batched=True, dedup=dedup)
    oe = oracle_run(oracle, prog, sr, facts, batched=True)
    gr, orr = ge.read("endpoints_connected"), oe.read("endpoints_connected")
    assert np.array_equal(gr["sample"], orr["sample"])
    if sr == "topk":
        assert_tags_close(gr["tags"], orr["prob"])
    elif sr == "diff_addmult":
        assert_tags_close(gr["tags"], orr["value"])
        gout = np.ones(orr["sample"].size, np.float32)
        ge.backward("endpoints_connected", gout)
        oe.backward("endpoints_connected", gout.astype(np.float64))
        n = g["src"].size
        np.testing.assert_allclose(ge.grad("edge", n), oe.grad("edge", n), rtol=1e-4, atol=1e-6)


@pytest.mark.parametrize("dedup", DEDUP)
def test_computed_value_outside_ids_is_an_error(synth, dedup):
    from paper_2503_21937_amd import dlfix
    src, dst, _ = synth.er_graph(1, 30, 60, weights=True)
    prog = ".input edge/2\nfar(x, y + 1000) :- edge(x, y).\n"
    e = dlfix.Engine(prog, "bool", dedup=dedup)
    e.add_facts("edge", [src, dst])
    with pytest.raises(dlfix.DLError) as ex:
        e.run()
    assert ex.value.status == 6  # DL_ERR_CAPACITY
