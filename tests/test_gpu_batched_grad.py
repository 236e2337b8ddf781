"""GPU parity of batched differentiable reachability on grids (add-mult with
reverse-mode gradients) against the CPU oracle and finite differences."""
import numpy as np
import pytest

from gpu_util import DEDUP, assert_tags_close, engine, oracle_run, same_rows

pytestmark = pytest.mark.gpu


def grid_facts(g, sel=None):
    if sel is None:
        sel = np.ones(g["src"].size, bool)
    return {"edge": ([g["src"][sel], g["dst"][sel]], g["p"][sel], g["sample"][sel])}


def query_grad(res, ks, samples):
    """grad_out = 1 on path(0, k^2 - 1) of every sample, 0 elsewhere (rows are
    in canonical (sample, x, z) order, so the query rows are found by search)."""
    key = (res["sample"].astype(np.int64) << 42) | (res["cols"][:, 0].astype(np.int64) << 21) \
        | res["cols"][:, 1].astype(np.int64)
    samples = np.asarray(list(samples), np.int64)
    want = (samples << 42) | (ks[samples].astype(np.int64) ** 2 - 1)
    i = np.searchsorted(key, want)
    assert np.array_equal(key[i], want)
    g = np.zeros(res["cols"].shape[0], np.float64)
    g[i] = 1.0
    return g


@pytest.mark.parametrize("dedup", DEDUP)
def test_small_batch_tags_and_grads_vs_oracle(oracle, synth, dedup):
    g = synth.grid_batch(3, samples=8, kmin=2, kmax=6)
    facts = grid_facts(g)
    ge = engine(synth.TC_PROGRAM, "diff_addmult", facts, batched=True, dedup=dedup)
    oe = oracle_run(oracle, synth.TC_PROGRAM, "diff_addmult", facts, batched=True)
    gr, orr = ge.read("path"), oe.read("path")
    same_rows(gr, orr, batched=True)
    assert_tags_close(gr["tags"], orr["value"])
    gout = query_grad(orr, g["ks"], range(8))
    ge.backward("path", gout.astype(np.float32))
    oe.backward("path", gout)
    gg = ge.grad("edge", g["src"].size)
    og = oe.grad("edge", g["src"].size)
    np.testing.assert_allclose(gg, og, rtol=1e-4, atol=1e-7)
    # and the oracle's reverse mode against central differences of its own
    # (pinned) binary64 forward, on a few edges
    rng = np.random.default_rng(0)
    for e in rng.choice(g["src"].size, 6, replace=False):
        h = 1e-3
        vals = []
        for sgn in (1, -1):
            p2 = g["p"].copy()
            p2[e] = np.float32(p2[e] + sgn * h)
            f2 = dict(edge=(facts["edge"][0], p2, facts["edge"][2]))
            r2 = oracle_run(oracle, synth.TC_PROGRAM, "diff_addmult", f2, batched=True).read("path")
            vals.append((float(gout @ r2["value"]), float(p2[e])))
        fd = (vals[0][0] - vals[1][0]) / (vals[0][1] - vals[1][1])
        assert gg[e] == pytest.approx(fd, rel=1e-3, abs=1e-6)


@pytest.mark.parametrize("dedup", DEDUP)
def test_batching_equals_separate_runs(synth, dedup):
    g = synth.grid_batch(5, samples=12, kmin=3, kmax=9)
    b = engine(synth.TC_PROGRAM, "diff_addmult", grid_facts(g), batched=True, dedup=dedup).read("path")
    for s in range(12):
        sel = g["sample"] == s
        one = engine(synth.TC_PROGRAM, "diff_addmult",
                     {"edge": ([g["src"][sel], g["dst"][sel]], g["p"][sel], None)}, dedup=dedup).read("path")
        m = b["sample"] == s
        assert np.array_equal(b["cols"][m], one["cols"])
        if dedup == "sort":
            assert np.array_equal(b["tags"][m], one["tags"])  # same +-order: identical
        else:  # float atomics: same terms, summation order may differ
            assert_tags_close(b["tags"][m], one["tags"], rtol=1e-6)


@pytest.mark.parametrize("dedup", DEDUP)
def test_full_size_sampled(oracle, synth, dedup):
    """512 grids, k ~ U{5..30}: the batched forward and the query gradient,
    checked per sample with the oracle's single-column solver."""
    g = synth.grid_batch(1)
    ge = engine(synth.TC_PROGRAM, "diff_addmult", grid_facts(g), batched=True, dedup=dedup)
    res = ge.read("path")
    ks = g["ks"]
    assert res["cols"].shape[0] == int((ks.astype(np.int64) ** 4).sum())  # grids: all pairs
    assert ge.stats()["max_rounds"] == 2 * (int(ks.max()) - 1) + 1
    gout = query_grad(res, ks, range(ks.size))
    ge.backward("path", gout.astype(np.float32))
    grad = ge.grad("edge", g["src"].size)
    rng = np.random.default_rng(1)
    picks = list(rng.choice(ks.size, 6, replace=False)) + [int(np.argmax(ks)), int(np.argmin(ks))]
    for s in picks:
        k = int(ks[s])
        sel = g["sample"] == s
        src, dst, p = g["src"][sel], g["dst"][sel], g["p"][sel]
        z = k * k - 1
        gc = np.zeros(k * k)
        gc[0] = 1.0
        col = oracle.tc_column(k * k, src, dst, p, "diff_addmult", z, grad_col=gc)
        m = (res["sample"] == s) & (res["cols"][:, 1] == z)
        assert np.array_equal(res["cols"][m, 0], np.arange(k * k))
        assert_tags_close(res["tags"][m], col["tag"], what=f"sample {s}")
        np.testing.assert_allclose(grad[sel], col["grad_edge"], rtol=2e-4, atol=1e-9)


def test_autograd_function(oracle, synth):
    import torch
    from paper_2503_21937_amd import dlfix
    from paper_2503_21937_amd.autograd import fixpoint
    g = synth.grid_batch(9, samples=6, kmin=3, kmax=7)
    e = dlfix.Engine(synth.TC_PROGRAM, "diff_addmult", batched=True)
    dev = torch.device("cuda")
    probs = torch.tensor(g["p"], device=dev, requires_grad=True)
    cols = [torch.tensor(g["src"].astype(np.int32), device=dev), torch.tensor(g["dst"].astype(np.int32), device=dev)]
    sample = torch.tensor(g["sample"].astype(np.int32), device=dev)
    tags, osample, ocols = fixpoint(probs, e, "edge", cols, sample, "path")
    ks = torch.tensor(g["ks"], device=dev)
    target = (ocols[:, 0] == 0) & (ocols[:, 1].long() == ks[osample.long()] ** 2 - 1)
    labels = torch.tensor(g["labels"], device=dev)
    pred = tags[target]
    loss = torch.nn.functional.binary_cross_entropy(pred.clamp(1e-6, 1 - 1e-6), labels[osample[target].long()])
    loss.backward()
    # the same gradient from the oracle, seeded with dloss/dtag
    with torch.no_grad():
        gout = torch.zeros_like(tags)
        pc = pred.clamp(1e-6, 1 - 1e-6)
        y = labels[osample[target].long()]
        gout[target] = (-(y / pc) + (1 - y) / (1 - pc)) / y.numel()
    o = oracle_run(oracle, synth.TC_PROGRAM, "diff_addmult", grid_facts(g), batched=True)
    o.backward("path", gout.cpu().double().numpy())
    want = o.grad("edge", g["src"].size)
    np.testing.assert_allclose(probs.grad.cpu().numpy(), want, rtol=1e-3, atol=1e-6)


def test_query_autograd_matches_full_read(synth):
    """Point lookups + row-seeded backward give the same loss gradient as
    reading the whole relation."""
    import torch
    from paper_2503_21937_amd import dlfix
    from paper_2503_21937_amd.autograd import fixpoint, fixpoint_query
    g = synth.grid_batch(11, samples=16, kmin=3, kmax=9)
    dev = torch.device("cuda")
    cols = [torch.tensor(g["src"].astype(np.int32), device=dev), torch.tensor(g["dst"].astype(np.int32), device=dev)]
    sample = torch.tensor(g["sample"].astype(np.int32), device=dev)
    ks = torch.tensor(g["ks"], device=dev)
    labels = torch.tensor(g["labels"], device=dev)
    S = int(g["ks"].size)
    # full read
    e1 = dlfix.Engine(synth.TC_PROGRAM, "diff_addmult", batched=True)
    p1 = torch.tensor(g["p"], device=dev, requires_grad=True)
    tags, osample, ocols = fixpoint(p1, e1, "edge", cols, sample, "path")
    target = (ocols[:, 0] == 0) & (ocols[:, 1].long() == ks[osample.long()] ** 2 - 1)
    pred1 = tags[target]
    loss1 = torch.nn.functional.binary_cross_entropy(pred1, labels[osample[target].long()], reduction="sum")
    loss1.backward()
    # queries only (plus one absent tuple: it reads as 0 and gets no gradient)
    e2 = dlfix.Engine(synth.TC_PROGRAM, "diff_addmult", batched=True)
    p2 = torch.tensor(g["p"], device=dev, requires_grad=True)
    qs = torch.arange(S, dtype=torch.int32, device=dev)
    qx = torch.zeros(S, dtype=torch.int32, device=dev)
    qz = (ks ** 2 - 1).to(torch.int32)
    pred2 = fixpoint_query(p2, e2, "edge", cols, sample, "path", [qx, qz], qs)
    assert torch.equal(pred2, pred1)
    loss2 = torch.nn.functional.binary_cross_entropy(pred2, labels, reduction="sum")
    loss2.backward()
    torch.testing.assert_close(p2.grad, p1.grad, rtol=1e-5, atol=1e-7)
    rows, t = e2.lookup("path", [np.array([0, 5000], np.uint32), np.array([1, 1], np.uint32)],
                        np.array([0, 0], np.uint32))
    assert rows[1] == -1 and t[1] == 0.0 and rows[0] >= 0
