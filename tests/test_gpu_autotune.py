"""The autotuner's candidate configurations all compute the oracle's
relation; its choice is cached and reused."""
import json
import os

import numpy as np
import pytest

from gpu_util import assert_tags_close, oracle_run

pytestmark = pytest.mark.gpu


def make_engine(synth, sr, src, dst, p):
    from paper_2503_21937_amd import dlfix
    e = dlfix.Engine(synth.TC_PROGRAM, sr)
    e.add_facts("edge", [src, dst], p)
    return e


@pytest.mark.parametrize("sr", ["maxmin", "minplus", "addmult", "bool"])
def test_every_configuration_matches_oracle(oracle, synth, sr, tmp_path):
    src, dst, p = synth.er_graph(5, 300, 1100, weights=True)
    want = oracle_run(oracle, synth.TC_PROGRAM, sr, {"edge": ([src, dst], p, None)}).read("path")
    key = _key(make_engine(synth, sr, src, dst, p))
    configs = [(dedup, orient, items, 1) for dedup in (1, 2) for orient in (1, 2) for items in (1, 2, 4, 8)]
    # row windows: off, and forced onto every launch they apply to
    configs += [(2, 2, items, rows) for items in (1, 4, 8) for rows in (0, 2)]
    for dedup, orient, items, rows in configs:
        e = make_engine(synth, sr, src, dst, p)
        cache = tmp_path / f"force_{sr}_{dedup}_{orient}_{items}_{rows}.jsonl"
        cache.write_text(json.dumps({"key": key, "dedup": dedup, "orient": orient, "items": items,
                                     "rows": rows, "ms": 1.0}) + "\n")
        cfg = e.autotune(1, str(cache))
        assert (cfg["dedup"], cfg["orient"], cfg["items"], cfg["rows"]) == (dedup, orient, items, rows)
        got = e.read("path")
        assert np.array_equal(got["cols"], want["cols"]), (dedup, orient, items, rows)
        if sr == "maxmin":
            assert np.array_equal(got["tags"].astype(np.float64), want["value"])
        elif sr in ("addmult", "minplus"):
            assert_tags_close(got["tags"], want["value"])


def _key(e):
    """The tuning key the library uses, read back through a throwaway cache."""
    import tempfile
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "c.jsonl")
        e.autotune(1, path)
        line = open(path).read().splitlines()[-1]
        return json.loads(line)["key"]


def test_autotune_picks_and_caches(oracle, synth, tmp_path):
    src, dst, p = synth.er_graph(1, 2000, 8000, weights=True)
    cache = str(tmp_path / "tune.jsonl")
    e = make_engine(synth, "minplus", src, dst, p)
    cfg = e.autotune(2, cache)
    assert cfg["tuned_ms"] > 0
    lines = open(cache).read().splitlines()
    assert len(lines) == 1
    rec = json.loads(lines[0])
    assert (rec["dedup"], rec["orient"], rec["items"]) == (cfg["dedup"], cfg["orient"], cfg["items"])
    e2 = make_engine(synth, "minplus", src, dst, p)
    cfg2 = e2.autotune(2, cache)  # served from the cache: no new line
    assert open(cache).read().splitlines() == lines
    assert (cfg2["dedup"], cfg2["orient"], cfg2["items"]) == (cfg["dedup"], cfg["orient"], cfg["items"])
    a, b = e.read("path"), e2.read("path")
    assert np.array_equal(a["cols"], b["cols"])
    assert np.array_equal(a["tags"], b["tags"])


@pytest.mark.parametrize("rows", [0, 1, 2])
def test_row_windows_batched(oracle, synth, tmp_path, rows):
    """Row windows keyed by (sample, first column) on a batch of grids (rows
    1: launches below the threshold take the row-window kernel's scattered
    fallback)."""
    from paper_2503_21937_amd import dlfix
    g = synth.grid_batch(9, samples=24, kmin=3, kmax=12)
    facts = {"edge": ([g["src"], g["dst"]], g["p"], g["sample"])}
    for sr in ("addmult", "maxmin", "bool", "diff_addmult"):
        e = dlfix.Engine(synth.TC_PROGRAM, sr, batched=True)
        e.add_facts("edge", [g["src"], g["dst"]], g["p"], g["sample"])
        key = _key(e)
        cache = tmp_path / f"rows_{sr}_{rows}.jsonl"
        cache.write_text(json.dumps({"key": key, "dedup": 2, "orient": 2, "items": 4, "rows": rows,
                                     "ms": 1.0}) + "\n")
        assert e.autotune(1, str(cache))["rows"] == rows
        got = e.read("path")
        o = oracle_run(oracle, synth.TC_PROGRAM, sr, facts, batched=True)
        want = o.read("path")
        assert np.array_equal(got["cols"], want["cols"]) and np.array_equal(got["sample"], want["sample"])
        if sr != "bool":
            assert_tags_close(got["tags"], want["value"])
        if sr == "diff_addmult":  # lineage logged by the row-window kernel
            gout = np.random.default_rng(4).normal(size=want["cols"].shape[0])
            e.backward("path", gout.astype(np.float32))
            o.backward("path", gout)
            np.testing.assert_allclose(e.grad("edge", g["src"].size), o.grad("edge", g["src"].size),
                                       rtol=1e-4, atol=1e-6)


@pytest.mark.parametrize("sr", ["maxmin", "addmult", "bool"])
def test_row_windows_hub_driver(oracle, synth, tmp_path, sr):
    """A driver group with more rows than the LDS row staging holds (a hub
    with 400 out-edges) takes the global-memory row search."""
    from paper_2503_21937_amd import dlfix
    rng = np.random.default_rng(12)
    n = 600
    src0, dst0, _ = synth.er_graph(12, n, 1500, weights=True)
    hub = np.zeros(400, np.uint32)
    hub_dst = rng.choice(np.arange(1, n, dtype=np.uint32), 400, replace=False)
    src = np.concatenate([src0, hub]).astype(np.uint32)
    dst = np.concatenate([dst0, hub_dst]).astype(np.uint32)
    p = rng.uniform(0.05, 0.9, src.size).astype(np.float32)
    e = make_engine(synth, sr, src, dst, p)
    key = _key(e)
    cache = tmp_path / "hub.jsonl"
    cache.write_text(json.dumps({"key": key, "dedup": 2, "orient": 2, "items": 2, "rows": 2, "ms": 1.0}) + "\n")
    assert e.autotune(1, str(cache))["rows"] == 2
    got = e.read("path")
    want = oracle_run(oracle, synth.TC_PROGRAM, sr, {"edge": ([src, dst], p, None)}).read("path")
    assert np.array_equal(got["cols"], want["cols"])
    if sr == "maxmin":
        assert np.array_equal(got["tags"].astype(np.float64), want["value"])
    elif sr == "addmult":
        assert_tags_close(got["tags"], want["value"])


SHAPES_PROGRAM = """
.input edge/2
.output hop/3
.output via/2
path(x, y) :- edge(x, y).
path(x, z) :- edge(x, y), path(y, z).
hop(x, y, z) :- edge(x, y), path(y, z).
via(x, y) :- edge(x, y), path(y, z).
"""


@pytest.mark.parametrize("rows", [1, 2])
@pytest.mark.parametrize("sr", ["maxmin", "minplus", "addmult", "bool"])
def test_row_windows_general_shapes(oracle, synth, tmp_path, sr, rows):
    """Row windows on heads the specialised variant does not take: a ternary
    head (window of n * np keys) and a binary head whose second column comes
    from the driver row; forced (rows 2) or by threshold (rows 1, where small
    launches take the kernel's scattered fallback)."""
    from paper_2503_21937_amd import dlfix
    src, dst, p = synth.er_graph(21, 60, 200, weights=True)
    e = dlfix.Engine(SHAPES_PROGRAM, sr)
    e.add_facts("edge", [src, dst], p)
    key = _key(e)
    cache = tmp_path / "shapes.jsonl"
    cache.write_text(json.dumps({"key": key, "dedup": 2, "orient": 2, "items": 2, "rows": rows, "ms": 1.0}) + "\n")
    assert e.autotune(1, str(cache))["rows"] == rows
    o = oracle_run(oracle, SHAPES_PROGRAM, sr, {"edge": ([src, dst], p, None)})
    for rel in ("path", "hop", "via"):
        got, want = e.read(rel), o.read(rel)
        assert np.array_equal(got["cols"], want["cols"]), rel
        if sr == "maxmin":
            assert np.array_equal(got["tags"].astype(np.float64), want["value"]), rel
        elif sr in ("addmult", "minplus"):
            assert_tags_close(got["tags"], want["value"], what=rel)
