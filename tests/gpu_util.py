"""Helpers shared by the GPU parity tests (HIP path through the C ABI vs the
CPU oracle on the same seeded inputs)."""
import numpy as np

TAG_RTOL = 1e-5  # float32 tags vs the binary64 oracle


DEDUP = ["sort", "dense"]  # both deduplication pipelines are parity-tested


def engine(program, semiring, facts, k=3, batched=False, dedup="auto", **kw):
    from paper_2503_21937_amd import dlfix
    e = dlfix.Engine(program, semiring, k=k, batched=batched, dedup=dedup, **kw)
    for rel, (cols, tags, sample) in facts.items():
        e.add_facts(rel, cols, tags, sample)
    return e.run()


def oracle_run(oracle, program, semiring, facts, k=3, batched=False):
    o = oracle.Oracle(program, semiring, k=k, batched=batched)
    for rel, (cols, tags, sample) in facts.items():
        o.add_facts(rel, cols, tags, sample)
    return o.run()


def assert_tags_close(got, want, rtol=TAG_RTOL, what=""):
    got = np.asarray(got, np.float64)
    want = np.asarray(want, np.float64)
    assert got.shape == want.shape, what
    both_inf = np.isinf(got) & np.isinf(want) & (np.sign(got) == np.sign(want))
    err = np.abs(got - want)
    bound = rtol * np.maximum(np.abs(got), np.abs(want)) + 1e-35
    bad = ~both_inf & ~(err <= bound)
    if bad.any():
        i = np.argmax(bad)
        raise AssertionError(f"{what}: {bad.sum()} tags differ, first at {i}: got {got[i]!r} want {want[i]!r}")


def same_rows(g, o, batched=False):
    """Tuple sets equal (bit-exact, canonical order)."""
    assert np.array_equal(g["cols"], o["cols"]), "tuple sets differ"
    if batched:
        assert np.array_equal(g["sample"], o["sample"]), "sample ids differ"


def tune_key(e):
    """The autotuner's key for an engine's current facts, read back through a
    throwaway cache (forcing a configuration then means writing that key)."""
    import json
    import os
    import tempfile
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "c.jsonl")
        e.autotune(1, path)
        line = open(path).read().splitlines()[-1]
        return json.loads(line)["key"]


def tc_closure(oracle, n, src, dst, p, sr, threads=16):
    """Transitive closure of a graph from the oracle's column solver (every
    target column evolves on its own in the naive rounds): (present[x, z],
    tag[x, z]) for all pairs.  Much faster than the generic evaluator."""
    import concurrent.futures as cf
    pres = np.zeros((n, n), bool)
    tag = np.zeros((n, n), np.float64)

    def col(z):
        c = oracle.tc_column(n, src, dst, None if sr == "bool" else p, sr, z)
        pres[:, z] = c["present"]
        tag[:, z] = c["tag"]

    with cf.ThreadPoolExecutor(threads) as ex:  # ctypes calls release the GIL
        list(ex.map(col, range(n)))
    return pres, tag


def check_closure(read, closure, sr, what=""):
    """A read `path` relation equals the closure: sets exact, max-min tags
    bit-exact, other float tags within TAG_RTOL."""
    pres, tag = closure
    cols = read["cols"]
    got = np.zeros(pres.shape, bool)
    got[cols[:, 0], cols[:, 1]] = True
    assert cols.shape[0] == int(pres.sum()), what
    assert np.array_equal(got, pres), what
    if sr == "bool":
        return
    want = tag[cols[:, 0], cols[:, 1]]
    if sr == "maxmin":
        assert np.array_equal(read["tags"].astype(np.float64), want), what
    else:
        assert_tags_close(read["tags"], want, what=what)
