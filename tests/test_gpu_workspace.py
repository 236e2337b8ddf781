"""The workspace contract of the C ABI: an engine given a block of device
memory (dl_options.workspace, here a torch tensor) keeps every device buffer
in it and never calls hipMalloc; a block that is too small gives
DL_ERR_NOMEM with the engine and its facts intact, and after
dl_set_workspace with a larger block the run matches the CPU oracle.

Every workspace here is filled with a non-zero byte pattern before use, and
blocks are reused by later engines, so a kernel that read memory it never
wrote (relying on zeroed fresh allocations) would show up as a parity
failure.
"""
import numpy as np
import pytest

from gpu_util import DEDUP, assert_tags_close, check_closure, oracle_run, same_rows, tc_closure

pytestmark = pytest.mark.gpu

NOMEM = 5
MIB = 1 << 20


def garbage(nbytes, byte=0xA5):
    import torch
    return torch.full((nbytes,), byte, dtype=torch.uint8, device="cuda")


def make(program, sr, facts, ws, **kw):
    from paper_2503_21937_amd import dlfix
    e = dlfix.Engine(program, sr, workspace=ws, **kw)
    for rel, (cols, tags, sample) in facts.items():
        e.add_facts(rel, cols, tags, sample)
    return e


@pytest.mark.parametrize("dedup", DEDUP)
@pytest.mark.parametrize("sr", ["bool", "maxmin", "minplus", "addmult"])
def test_tc_in_dirty_workspace(oracle, synth, sr, dedup):
    src, dst, p = synth.er_graph(2, 1000, 4000, weights=True)
    facts = {"edge": ([src, dst], None if sr == "bool" else p, None)}
    e = make(synth.TC_PROGRAM, sr, facts, garbage(512 * MIB), dedup=dedup)
    e.run()
    want = tc_closure(oracle, 1000, src, dst, p, sr)
    check_closure(e.read("path"), want, sr)
    st = e.stats()
    assert st["device_allocs"] == 0
    assert 0 < st["workspace_peak"] <= 512 * MIB
    # a second run on the same engine reuses the ranges it holds
    e.run()
    check_closure(e.read("path"), want, sr)
    assert e.stats()["device_allocs"] == 0


@pytest.mark.parametrize("dedup", DEDUP)
def test_too_small_then_larger(oracle, synth, dedup):
    src, dst, p = synth.er_graph(3, 1500, 6000, weights=True)
    facts = {"edge": ([src, dst], p, None)}
    from paper_2503_21937_amd import dlfix
    e = make(synth.TC_PROGRAM, "maxmin", facts, garbage(2 * MIB), dedup=dedup)
    with pytest.raises(dlfix.DLError) as ex:
        e.run()
    assert ex.value.status == NOMEM
    assert "workspace" in str(ex.value)
    with pytest.raises(dlfix.DLError) as ex:  # still too small: the same answer, nothing lost
        e.run()
    assert ex.value.status == NOMEM
    e.set_workspace(garbage(1024 * MIB, 0x3C))
    e.run()
    check_closure(e.read("path"), tc_closure(oracle, 1500, src, dst, p, "maxmin"), "maxmin")
    assert e.stats()["device_allocs"] == 0


def test_move_keeps_results(oracle, synth):
    """Results and facts survive moves: workspace -> library allocations ->
    another workspace, read after each move; then a rerun."""
    src, dst, p = synth.er_graph(1, 700, 2800, weights=True)
    facts = {"edge": ([src, dst], p, None)}
    e = make(synth.TC_PROGRAM, "minplus", facts, garbage(256 * MIB))
    e.run()
    want = tc_closure(oracle, 700, src, dst, p, "minplus")
    check_closure(e.read("path"), want, "minplus")
    e.set_workspace(None)
    check_closure(e.read("path"), want, "minplus")
    allocs = e.stats()["device_allocs"]
    assert allocs > 0
    e.set_workspace(garbage(256 * MIB, 0x5A))
    check_closure(e.read("path"), want, "minplus")
    e.run()
    check_closure(e.read("path"), want, "minplus")
    assert e.stats()["device_allocs"] == allocs  # no allocation since the last move


def test_block_reused_by_next_engine(oracle, synth):
    """One block serves engines one after another (the previous one freed):
    the second engine starts from the first one's leftovers."""
    ws = garbage(512 * MIB)
    for seed, sr in ((1, "maxmin"), (2, "addmult"), (3, "bool")):
        src, dst, p = synth.er_graph(seed, 900, 3600, weights=True)
        facts = {"edge": ([src, dst], None if sr == "bool" else p, None)}
        e = make(synth.TC_PROGRAM, sr, facts, ws)
        e.run()
        check_closure(e.read("path"), tc_closure(oracle, 900, src, dst, p, sr), sr)
        e.close()


@pytest.mark.parametrize("dedup", DEDUP)
def test_batched_grads_in_workspace(oracle, synth, dedup):
    """Diff add-mult on a batch of grids, forward and reverse pass, lineage
    recorded and recomputed, all inside a dirty workspace."""
    g = synth.grid_batch(4, samples=16, kmin=3, kmax=9)
    facts = {"edge": ([g["src"], g["dst"]], g["p"], g["sample"])}
    o = oracle_run(oracle, synth.TC_PROGRAM, "diff_addmult", facts, batched=True)
    orr = o.read("path")
    gout = synth.normal_grads(7, orr["cols"].shape[0])
    o.backward("path", gout.astype(np.float64))
    og = o.grad("edge", g["src"].size)
    for lineage in ("store", "recompute"):
        e = make(synth.TC_PROGRAM, "diff_addmult", facts, garbage(64 * MIB), batched=True, dedup=dedup,
                 lineage=lineage)
        e.run()
        gr = e.read("path")
        same_rows(gr, orr, batched=True)
        assert_tags_close(gr["tags"], orr["value"])
        e.backward("path", gout)
        np.testing.assert_allclose(e.grad("edge", g["src"].size), og, rtol=1e-4, atol=1e-6)
        assert e.stats()["device_allocs"] == 0


def test_topk_in_workspace(oracle, synth):
    from test_gpu_topk import RELS, scene_facts
    sc = synth.topk_scenes(5, samples=24)
    facts = scene_facts(sc)
    e = make(synth.TOPK_PROGRAM, "diff_topk", facts, garbage(32 * MIB), k=3, batched=True)
    e.run()
    o = oracle_run(oracle, synth.TOPK_PROGRAM, "diff_topk", facts, k=3, batched=True)
    for rel in ("q", "reach"):
        gr, orr = e.read(rel), o.read(rel)
        same_rows(gr, orr, batched=True)
        assert np.array_equal(gr["bits"], orr["bits"]), rel
        assert_tags_close(gr["tags"], orr["prob"], what=rel)
    n = o.size("reach")
    gout = synth.normal_grads(2, n)
    e.backward("reach", gout)
    o.backward("reach", gout.astype(np.float64))
    for r in RELS:
        n = facts[r][0][0].size
        np.testing.assert_allclose(e.grad(r, n), o.grad(r, n), rtol=1e-4, atol=1e-6, err_msg=r)
    assert e.stats()["device_allocs"] == 0


@pytest.mark.parametrize("dedup", DEDUP)
def test_points_to_in_workspace(oracle, synth, dedup):
    rels = synth.andersen(1, v=600, n_addr=300, n_assign=1800, n_load=240, n_store=240)
    facts = {name: ([a, b], None, None) for name, (a, b) in rels.items()}
    e = make(synth.ANDERSEN_PROGRAM, "bool", facts, garbage(256 * MIB), dedup=dedup)
    e.run()
    o = oracle_run(oracle, synth.ANDERSEN_PROGRAM, "bool", facts)
    assert np.array_equal(e.read("pt")["cols"], o.read("pt")["cols"])
    assert e.stats()["device_allocs"] == 0


def test_autograd_regrows_its_workspace(oracle, synth):
    """The autograd wrapper doubles a workspace tensor that is too small and
    runs again; the result equals the oracle's."""
    import torch
    from paper_2503_21937_amd import autograd, dlfix
    g = synth.grid_batch(6, samples=8, kmin=4, kmax=8)
    facts = {"edge": ([g["src"], g["dst"]], g["p"], g["sample"])}
    e = dlfix.Engine(synth.TC_PROGRAM, "diff_addmult", batched=True, workspace=garbage(1 * MIB))
    probs = torch.tensor(g["p"], device="cuda", requires_grad=True)
    cols = [torch.tensor(g["src"].astype(np.int32), device="cuda"),
            torch.tensor(g["dst"].astype(np.int32), device="cuda")]
    sample = torch.tensor(g["sample"].astype(np.int32), device="cuda")
    tags, _, _ = autograd.fixpoint(probs, e, "edge", cols, sample)
    assert e.workspace.nbytes > 1 * MIB
    orr = oracle_run(oracle, synth.TC_PROGRAM, "diff_addmult", facts, batched=True).read("path")
    assert_tags_close(tags.detach().cpu().numpy(), orr["value"])
    tags.sum().backward()
    assert torch.isfinite(probs.grad).all()
    assert e.stats()["device_allocs"] == 0
