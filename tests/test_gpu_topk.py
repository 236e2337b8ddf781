"""GPU parity of batched top-k proofs (3-way join + recursive rule) and the
gradient of the proof probabilities, against the CPU oracle."""
import numpy as np
import pytest

from gpu_util import assert_tags_close, engine, oracle_run, same_rows

pytestmark = pytest.mark.gpu

RELS = [f"u{i}" for i in range(8)] + [f"r{i}" for i in range(4)]


def scene_facts(sc):
    f = {}
    for r in RELS:
        if r[0] == "u":
            s, a, p = sc[r]
            f[r] = ([a], p, s)
        else:
            s, a, b, p = sc[r]
            f[r] = ([a, b], p, s)
    return f


@pytest.mark.parametrize("k", [1, 3])
@pytest.mark.parametrize("samples", [8, 256])
def test_topk_scenes(oracle, synth, k, samples):
    sc = synth.topk_scenes(2, samples=samples)
    facts = scene_facts(sc)
    ge = engine(synth.TOPK_PROGRAM, "diff_topk", facts, k=k, batched=True)
    oe = oracle_run(oracle, synth.TOPK_PROGRAM, "diff_topk", facts, k=k, batched=True)
    for rel in ("q", "reach"):
        gr, orr = ge.read(rel), oe.read(rel)
        same_rows(gr, orr, batched=True)
        assert np.array_equal(gr["cnt"].astype(np.int32), orr["cnt"])
        assert np.array_equal(gr["bits"][:, :k], orr["bits"][:, :k]), rel
        assert np.array_equal(gr["p"][:, :k], orr["p"][:, :k]), rel  # same binary32 products
        assert_tags_close(gr["tags"], orr["prob"], what=rel)
    # gradient of sum_t g_t P(t) over both output relations
    for rel, seed in (("q", 3), ("reach", 4)):
        n = oe.size(rel)
        gout = synth.normal_grads(seed, n)
        ge.backward(rel, gout)
        oe.backward(rel, gout.astype(np.float64))
    for r in RELS:
        n = facts[r][0][0].size
        np.testing.assert_allclose(ge.grad(r, n), oe.grad(r, n), rtol=1e-4, atol=1e-6, err_msg=r)


def test_proof_overflow(synth):
    """A sample may hold 256 probabilistic facts (four-word proof sets), not 257."""
    from paper_2503_21937_amd import dlfix
    e = dlfix.Engine(synth.TC_PROGRAM, "topk")
    src = np.arange(257, dtype=np.uint32)
    e.add_facts("edge", [src[:256], src[:256] + 1], np.full(256, 0.5, np.float32))
    with pytest.raises(dlfix.DLError) as ex:
        e.add_facts("edge", [src[256:], src[256:] + 1], np.full(1, 0.5, np.float32))
    assert ex.value.status == 7
