"""GPU parity of the transitive-closure fixpoint (HIP path vs CPU oracle)."""
import numpy as np
import pytest

from gpu_util import DEDUP, assert_tags_close, engine, oracle_run, same_rows

pytestmark = pytest.mark.gpu

SEMIRINGS = ["bool", "maxmin", "minplus", "addmult"]


def tc_facts(src, dst, p, sample=None):
    return {"edge": ([src, dst], p, sample)}


def check_tc(oracle, synth, src, dst, p, sr, rounds=True, dedup="auto"):
    facts = tc_facts(src, dst, None if sr == "bool" else p)
    g = engine(synth.TC_PROGRAM, sr, facts, dedup=dedup)
    o = oracle_run(oracle, synth.TC_PROGRAM, sr, facts)
    gr, orr = g.read("path"), o.read("path")
    same_rows(gr, orr)
    if sr == "maxmin":
        assert np.array_equal(gr["tags"].astype(np.float64), orr["value"])
    elif sr != "bool":
        assert_tags_close(gr["tags"], orr["value"], what=sr)
    if rounds and sr != "minplus":  # min-plus: binary32 vs binary64 ties may move a round
        assert g.stats()["max_rounds"] == o.rounds()
    return g, gr


@pytest.mark.parametrize("dedup", DEDUP)
@pytest.mark.parametrize("seed", [1, 2, 3])
@pytest.mark.parametrize("sr", SEMIRINGS)
def test_er256_parity(oracle, synth, sr, seed, dedup):
    src, dst, p = synth.er_graph(seed, 256, 1024, weights=True)
    check_tc(oracle, synth, src, dst, p, sr, dedup=dedup)


@pytest.mark.parametrize("dedup", DEDUP)
@pytest.mark.parametrize("sr", SEMIRINGS)
def test_edge_cases(oracle, synth, sr, dedup):
    cases = [
        ([0], [1]),                       # one edge
        ([0, 1], [1, 0]),                 # 2-cycle: reflexive paths appear
        ([3], [3]),                       # self loop
        ([0, 1, 2, 3, 4], [1, 2, 3, 4, 0]),  # directed 5-cycle
        (list(range(199)), list(range(1, 200))),  # long chain: 200 rounds
    ]
    rng = np.random.default_rng(0)
    for s, d in cases:
        s = np.asarray(s, np.uint32)
        d = np.asarray(d, np.uint32)
        p = synth.unit_prob(rng, s.size)
        check_tc(oracle, synth, s, d, p, sr, dedup=dedup)


@pytest.mark.parametrize("dedup", DEDUP)
def test_duplicate_facts_are_merged(oracle, synth, dedup):
    src = np.array([0, 0, 1, 1, 2], np.uint32)
    dst = np.array([1, 1, 2, 2, 0], np.uint32)
    p = np.array([0.25, 0.5, 0.125, 0.5, 0.75], np.float32)
    for sr in SEMIRINGS:
        check_tc(oracle, synth, src, dst, p, sr, dedup=dedup)


@pytest.mark.parametrize("dedup", DEDUP)
def test_no_facts(synth, dedup):
    from paper_2503_21937_amd import dlfix
    e = dlfix.Engine(synth.TC_PROGRAM, "addmult", dedup=dedup).run()
    assert e.size("path") == 0
    assert e.stats()["rounds"] == 1


@pytest.mark.parametrize("dedup", DEDUP)
@pytest.mark.parametrize("sr", SEMIRINGS)
def test_er2000_multi_tile(oracle, synth, sr, dedup):
    """Multi-tile sizes with ragged tails: every join/sort/merge spans many
    workgroups.  Checked column by column against the oracle."""
    n = 2000
    src, dst, p = synth.er_graph(7, n, 7000, weights=True)
    g = engine(synth.TC_PROGRAM, sr, tc_facts(src, dst, None if sr == "bool" else p), dedup=dedup)
    r = g.read("path")
    cols = r["cols"]
    for z in range(3, n, 97):
        c = oracle.tc_column(n, src, dst, p, sr, z)
        m = cols[:, 1] == z
        assert np.array_equal(cols[m, 0], np.nonzero(c["present"])[0]), z
        if sr == "maxmin":
            assert np.array_equal(r["tags"][m].astype(np.float64), c["tag"][cols[m, 0]])
        elif sr != "bool":
            assert_tags_close(r["tags"][m], c["tag"][cols[m, 0]], what=f"{sr} z={z}")


@pytest.mark.parametrize("dedup", DEDUP)
def test_determinism(synth, dedup):
    src, dst, p = synth.er_graph(2, 256, 1024, weights=True)
    for sr in ["bool", "maxmin", "minplus"]:
        a = engine(synth.TC_PROGRAM, sr, tc_facts(src, dst, p), dedup=dedup).read("path")
        b = engine(synth.TC_PROGRAM, sr, tc_facts(src, dst, p), dedup=dedup).read("path")
        assert np.array_equal(a["cols"], b["cols"])
        assert np.array_equal(a["tags"].view(np.uint32), b["tags"].view(np.uint32))


def test_device_pointers_roundtrip(oracle, synth):
    import torch
    src, dst, p = synth.er_graph(1, 256, 1024, weights=True)
    from paper_2503_21937_amd import dlfix
    e = dlfix.Engine(synth.TC_PROGRAM, "maxmin")
    t = lambda a, dt: torch.from_numpy(a.astype(dt)).cuda()
    e.add_facts("edge", [t(src, np.int32), t(dst, np.int32)], t(p, np.float32))
    e.run()
    r = e.read("path", device=True)
    torch.cuda.synchronize()
    o = oracle_run(oracle, synth.TC_PROGRAM, "maxmin", tc_facts(src, dst, p)).read("path")
    cols = np.stack([c.cpu().numpy().astype(np.uint32) for c in r["cols"]], 1)
    assert np.array_equal(cols, o["cols"])
    assert np.array_equal(r["tags"].cpu().numpy().astype(np.float64), o["value"])


def test_dedup_pipelines_agree(synth):
    """The sort-based and the dense-domain pipelines give the same relation."""
    src, dst, p = synth.er_graph(4, 3000, 12000, weights=True)
    for sr in SEMIRINGS:
        a = engine(synth.TC_PROGRAM, sr, tc_facts(src, dst, p), dedup="sort")
        b = engine(synth.TC_PROGRAM, sr, tc_facts(src, dst, p), dedup="dense")
        ra, rb = a.read("path"), b.read("path")
        assert np.array_equal(ra["cols"], rb["cols"]), sr
        if sr in ("maxmin", "minplus", "bool"):
            assert np.array_equal(ra["tags"], rb["tags"]), sr
        else:
            assert_tags_close(ra["tags"], rb["tags"], rtol=1e-6, what=sr)
        assert a.stats()["max_rounds"] == b.stats()["max_rounds"], sr


def test_graph_replay_matches_eager_rounds(synth):
    """Round bodies replayed from a captured HIP graph give the relation the
    eagerly launched rounds give, on repeated runs of one engine with other
    GPU work and synchronisations in between."""
    import torch
    from paper_2503_21937_amd import dlfix
    src, dst, p = synth.er_graph(6, 3000, 12000, weights=True)
    for sr in SEMIRINGS:
        eager = dlfix.Engine(synth.TC_PROGRAM, sr, graphs=False)
        eager.add_facts("edge", [src, dst], p)
        ref = eager.run().read("path")
        g = dlfix.Engine(synth.TC_PROGRAM, sr, graphs=True)
        g.add_facts("edge", [src, dst], p)
        for rep in range(3):
            x = torch.randn(1 << 20, device="cuda")
            (x * 2).sum().item()
            got = g.run().read("path")
            torch.cuda.synchronize()
            assert np.array_equal(got["cols"], ref["cols"]), (sr, rep)
            if sr == "addmult":
                assert_tags_close(got["tags"], ref["tags"], rtol=1e-6, what=sr)
            else:
                assert np.array_equal(got["tags"], ref["tags"]), (sr, rep)
            assert g.stats()["max_rounds"] == eager.stats()["max_rounds"]


JOIN2 = ".input a/2\n.input b/2\n.output c/2\nc(x, z) :- a(x, y), b(y, z).\n"


@pytest.mark.parametrize("dedup", DEDUP)
@pytest.mark.parametrize("sr", ["bool", "maxmin"])
@pytest.mark.parametrize("n", [1, 255, 256, 257, 513, 70000])
def test_join_counts_across_tiles(oracle, sr, dedup, n):
    """Single-pass count + scan: probe-row counts at and around multiples of
    its 256-row tiles (one tile, a tile and one row, many tiles)."""
    rng = np.random.default_rng(n)
    ax = rng.integers(0, 400, n).astype(np.uint32)
    ay = rng.integers(0, 300, n).astype(np.uint32)
    bx = rng.integers(0, 300, 900).astype(np.uint32)
    bz = rng.integers(0, 400, 900).astype(np.uint32)
    pa = rng.uniform(0.1, 0.9, n).astype(np.float32) if sr != "bool" else None
    pb = rng.uniform(0.1, 0.9, 900).astype(np.float32) if sr != "bool" else None
    facts = {"a": ([ax, ay], pa, None), "b": ([bx, bz], pb, None)}
    g = engine(JOIN2, sr, facts, dedup=dedup).read("c")
    o = oracle_run(oracle, JOIN2, sr, facts).read("c")
    same_rows(g, o)
    if sr == "maxmin":
        assert np.array_equal(g["tags"].astype(np.float64), o["value"])


@pytest.mark.parametrize("dedup", DEDUP)
@pytest.mark.parametrize("n", [2048 * 256 + 1, 8192 * 256])
def test_join_counts_many_tiles(dedup, n):
    """Single-pass count + scan at its largest sizes (2049 and 8192 tiles of
    256 distinct probe rows), checked against the boolean and max-min matrix
    products computed here (c = a o b)."""
    from scipy.sparse import csr_matrix
    rng = np.random.default_rng(n)
    nx, ny, nz = 8192, 300, 400
    cell = rng.choice(nx * ny, size=n, replace=False)
    ax, ay = (cell // ny).astype(np.uint32), (cell % ny).astype(np.uint32)
    bcell = rng.choice(ny * nz, size=900, replace=False)
    bx, bz = (bcell // nz).astype(np.uint32), (bcell % nz).astype(np.uint32)
    pa = rng.uniform(0.1, 0.9, n).astype(np.float32)
    pb = rng.uniform(0.1, 0.9, 900).astype(np.float32)
    facts = {"a": ([ax, ay], pa, None), "b": ([bx, bz], pb, None)}
    A = csr_matrix((np.ones(n), (ax, ay)), shape=(nx, ny))
    B = csr_matrix((np.ones(900), (bx, bz)), shape=(ny, nz))
    want = np.argwhere((A @ B).toarray() > 0).astype(np.uint32)
    g = engine(JOIN2, "bool", facts, dedup=dedup).read("c")
    assert np.array_equal(g["cols"], want)
    # max-min: c(x, z) = max over y of min(a(x, y), b(y, z)), by rows of b
    C = np.zeros((nx, nz), np.float64)
    for y, z, q in zip(bx, bz, pb.astype(np.float64)):
        m = ay == y
        np.maximum.at(C[:, z], ax[m], np.minimum(pa[m].astype(np.float64), q))
    g = engine(JOIN2, "maxmin", facts, dedup=dedup).read("c")
    assert np.array_equal(g["cols"], want)
    assert np.array_equal(g["tags"].astype(np.float64), C[want[:, 0], want[:, 1]])
