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
