"""Kernel timing (dl_profile): a timed run gives the same relation as an
untimed one, and engines built with and without round graphs (timed rounds
are launched directly) report the same launches and algorithmic bytes per
family (with rounds fused into one launch and without), and so does a second
timed run of the same engine."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("fused", [True, False])
@pytest.mark.parametrize("sr", ["maxmin", "addmult"])
def test_profiled_graphs_match_direct_launches(synth, sr, fused):
    from paper_2503_21937_amd import dlfix
    src, dst, p = synth.er_graph(3, 1500, 6000, weights=True)
    runs = {}
    for graphs in (True, False):
        e = dlfix.Engine(synth.TC_PROGRAM, sr, dedup="dense", graphs=graphs, fused=fused)
        e.add_facts("edge", [src, dst], p)
        plain = e.run().read("path")
        e.profile(["join_expand", "join_count"])
        timed = e.run().read("path")
        ks = e.kernel_stats()
        assert np.array_equal(plain["cols"], timed["cols"])
        assert np.array_equal(plain["tags"], timed["tags"]) or sr == "addmult"
        runs[graphs] = (timed, ks)
        # a second timed run (round graphs kept from the first) counts the same
        e.profile(["join_expand", "join_count"])
        e.run()
        ks2 = e.kernel_stats()
        for fam in ("join_expand", "join_count"):
            assert ks2[fam]["launches"] == ks[fam]["launches"], fam
            assert ks2[fam]["bytes"] == pytest.approx(ks[fam]["bytes"], rel=1e-9), fam
        # and a family no longer timed is not counted
        e.profile(["join_count"])
        e.run()
        assert e.kernel_stats()["join_expand"]["launches"] == 0
    (g, kg), (d, kd) = runs[True], runs[False]
    assert np.array_equal(g["cols"], d["cols"])
    # fused rounds count the matches inside the join launch
    fams = ("join_expand",) if fused else ("join_expand", "join_count")
    for fam in fams:
        assert kg[fam]["launches"] == kd[fam]["launches"] > 0, fam
        assert kg[fam]["ms"] > 0 and kd[fam]["ms"] > 0, fam
        assert kg[fam]["bytes"] == pytest.approx(kd[fam]["bytes"], rel=1e-9), fam
    if fused:
        assert kg["join_count"]["launches"] == kd["join_count"]["launches"] == 0


@pytest.mark.parametrize("dedup", ["sort", "hash"])
def test_round_log_sort_path(oracle, synth, dedup):
    """Every round of the sort path is logged with its derivations (counted
    on the host), and the new tuples add up to the relation."""
    from paper_2503_21937_amd import dlfix
    src, dst, p = synth.er_graph(6, 400, 1200, weights=True)
    e = dlfix.Engine(synth.TC_PROGRAM, "addmult", dedup=dedup)
    e.add_facts("edge", [src, dst], p)
    e.run()
    log = e.round_log()
    st = e.stats()
    assert log["kind"].size == st["max_rounds"]
    assert log["kind"][0] == 1 and np.all(log["kind"][1:] == 2)
    assert int(log["derivations"].sum()) == st["candidates"]
    assert int(log["new"].sum()) == e.size("path")  # frozen tags: every tuple is new once
    assert log["new"][-1] == 0
