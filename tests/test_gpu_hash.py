"""GPU parity of the hash-index joins (open addressing, linear probing, one
slot per distinct join prefix with its first row and row count) against the
CPU oracle: forced through the autotuner's cache on the transitive closure
under every semiring and both deduplication pipelines, on batched samples,
and taken by themselves where the join prefix domain is wider than CSR
offsets can cover (two 17-bit join columns)."""
import json

import numpy as np
import pytest

from gpu_util import assert_tags_close, check_closure, engine, oracle_run, same_rows, tc_closure, tune_key

pytestmark = pytest.mark.gpu


def force(e, tmp_path, dedup, orient=1, items=2, rows=1, index=1):
    key = tune_key(e)
    cache = tmp_path / "force.jsonl"
    cache.write_text(json.dumps({"key": key, "dedup": dedup, "orient": orient, "items": items, "rows": rows,
                                 "index": index, "ms": 1.0}) + "\n")
    e.autotune(1, str(cache))
    assert e.stats()["index"] == index


@pytest.mark.parametrize("dedup", [1, 2])
@pytest.mark.parametrize("sr", ["bool", "maxmin", "minplus", "addmult"])
def test_tc_hash_index(oracle, synth, sr, dedup, tmp_path):
    from paper_2503_21937_amd import dlfix
    n, m = 800, 3200
    src, dst, p = synth.er_graph(7, n, m, weights=True)
    e = dlfix.Engine(synth.TC_PROGRAM, sr)
    e.add_facts("edge", [src, dst], None if sr == "bool" else p)
    force(e, tmp_path, dedup)
    check_closure(e.read("path"), tc_closure(oracle, n, src, dst, p, sr), sr, f"hash dedup={dedup}")


@pytest.mark.parametrize("sr", ["maxmin", "addmult"])
def test_batched_hash_index(oracle, synth, sr, tmp_path):
    from paper_2503_21937_amd import dlfix
    g = synth.grid_batch(4, samples=16, kmin=3, kmax=10)
    facts = {"edge": ([g["src"], g["dst"]], g["p"], g["sample"])}
    e = dlfix.Engine(synth.TC_PROGRAM, sr, batched=True)
    e.add_facts("edge", [g["src"], g["dst"]], g["p"], g["sample"])
    force(e, tmp_path, 1)
    o = oracle_run(oracle, synth.TC_PROGRAM, sr, facts, batched=True)
    gr, orr = e.read("path"), o.read("path")
    same_rows(gr, orr, batched=True)
    assert_tags_close(gr["tags"], orr["value"])


WIDE = """
.input e/3
.input f/3
r(x, y, z) :- e(x, y, z).
r(x, y, w) :- r(x, z, y), f(z, y, w).
"""


@pytest.mark.parametrize("sr", ["bool", "maxmin"])
def test_prefix_wider_than_csr(oracle, sr):
    """f is indexed on two 17-bit columns: a 34-bit prefix domain, which only
    the hash index covers (CSR offsets stop at 2^30)."""
    rng = np.random.default_rng(11)
    pool = rng.choice(1 << 17, 150, replace=False).astype(np.uint32)
    ne, nf = 400, 1500
    e_cols = [pool[rng.integers(0, 150, ne)] for _ in range(3)]
    f_cols = [pool[rng.integers(0, 150, nf)] for _ in range(3)]
    facts = {"e": (e_cols, rng.uniform(0.1, 0.9, ne).astype(np.float32) if sr != "bool" else None, None),
             "f": (f_cols, rng.uniform(0.1, 0.9, nf).astype(np.float32) if sr != "bool" else None, None)}
    g = engine(WIDE, sr, facts)
    assert g.stats()["id_bits"] == 17
    o = oracle_run(oracle, WIDE, sr, facts)
    gr, orr = g.read("r"), o.read("r")
    same_rows(gr, orr)
    assert gr["cols"].shape[0] > ne  # the recursive rule derived tuples
    if sr == "maxmin":
        assert np.array_equal(gr["tags"].astype(np.float64), orr["value"])
    assert g.stats()["max_rounds"] == o.rounds()


def test_autotuner_records_index(synth, tmp_path):
    from paper_2503_21937_amd import dlfix
    src, dst, p = synth.er_graph(2, 300, 1200, weights=True)
    e = dlfix.Engine(synth.TC_PROGRAM, "maxmin")
    e.add_facts("edge", [src, dst], p)
    cache = tmp_path / "t.jsonl"
    e.autotune(1, str(cache))
    rec = json.loads(cache.read_text().splitlines()[-1])
    assert rec["index"] in (0, 1) and rec["index"] == e.stats()["index"]


# ------------------------------------------------ hash-set deduplication

@pytest.mark.parametrize("sr", ["bool", "maxmin", "minplus", "addmult"])
def test_tc_hash_set(oracle, synth, sr):
    """Each round's candidates deduplicated in a hash set (tags folded per
    key with atomics), then only the distinct keys sorted."""
    from paper_2503_21937_amd import dlfix
    n, m = 900, 3600
    src, dst, p = synth.er_graph(8, n, m, weights=True)
    e = dlfix.Engine(synth.TC_PROGRAM, sr, dedup="hash")
    e.add_facts("edge", [src, dst], None if sr == "bool" else p)
    e.run()
    assert e.stats()["dedup"] == 3
    check_closure(e.read("path"), tc_closure(oracle, n, src, dst, p, sr), sr, "hash set")


NONLINEAR = ".input edge/2\npath(x, y) :- edge(x, y).\npath(x, z) :- path(x, y), path(y, z).\n"


@pytest.mark.parametrize("sr", ["maxmin", "addmult"])
def test_nonlinear_and_batched_hash_set(oracle, synth, sr):
    src, dst, p = synth.er_graph(3, 300, 900, weights=True)
    facts = {"edge": ([src, dst], p, None)}
    g = engine(NONLINEAR, sr, facts, dedup="hash")
    o = oracle_run(oracle, NONLINEAR, sr, facts)
    gr, orr = g.read("path"), o.read("path")
    same_rows(gr, orr)
    assert_tags_close(gr["tags"], orr["value"])
    gb = synth.grid_batch(6, samples=12, kmin=3, kmax=9)
    facts = {"edge": ([gb["src"], gb["dst"]], gb["p"], gb["sample"])}
    g = engine(synth.TC_PROGRAM, sr, facts, batched=True, dedup="hash")
    o = oracle_run(oracle, synth.TC_PROGRAM, sr, facts, batched=True)
    gr, orr = g.read("path"), o.read("path")
    same_rows(gr, orr, batched=True)
    assert_tags_close(gr["tags"], orr["value"])
    assert g.stats()["max_rounds"] == o.rounds()


def test_hash_set_with_wide_keys_and_points_to(oracle, synth):
    """64-bit packed keys (three 17-bit columns) and three-atom rules."""
    rng = np.random.default_rng(12)
    pool = rng.choice(1 << 17, 120, replace=False).astype(np.uint32)
    facts = {"e": ([pool[rng.integers(0, 120, 300)] for _ in range(3)], None, None),
             "f": ([pool[rng.integers(0, 120, 1200)] for _ in range(3)], None, None)}
    g = engine(WIDE, "bool", facts, dedup="hash")
    assert g.stats()["key_bits"] == 64
    o = oracle_run(oracle, WIDE, "bool", facts)
    same_rows(g.read("r"), o.read("r"))
    rels = synth.andersen(4, v=500, n_addr=250, n_assign=1500, n_load=200, n_store=200)
    facts = {name: ([a, b], None, None) for name, (a, b) in rels.items()}
    g = engine(synth.ANDERSEN_PROGRAM, "bool", facts, dedup="hash")
    o = oracle_run(oracle, synth.ANDERSEN_PROGRAM, "bool", facts)
    assert np.array_equal(g.read("pt")["cols"], o.read("pt")["cols"])
