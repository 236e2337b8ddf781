"""dl_load_program_static: the entry point for callers that cannot allocate.
Its engines keep every device buffer in the library's static per-device
array; their results must equal those of dl_load_program's engines (and the
oracle's), call after call, including a second call with a smaller input,
with no allocation at all."""
import numpy as np
import pytest

from gpu_util import check_closure, tc_closure

pytestmark = pytest.mark.gpu

STATIC_BYTES = 128 << 20  # DL_STATIC_WORKSPACE_MIB
STATE, NOMEM = 4, 5


def tc_engine(synth, src, dst, p, sr, static):
    from paper_2503_21937_amd import dlfix
    e = dlfix.Engine(synth.TC_PROGRAM, sr, static=static)
    e.add_facts("edge", [src, dst], None if sr == "bool" else p)
    return e.run()


def same(a, b, sr):
    assert np.array_equal(a["cols"], b["cols"]), sr
    if sr in ("bool", "maxmin"):
        assert np.array_equal(a["tags"], b["tags"]), sr  # exact: no rounding in max / min
    else:  # add-mult sums are folded with float atomics: equal up to rounding order
        np.testing.assert_allclose(a["tags"], b["tags"], rtol=1e-5, err_msg=sr)


@pytest.mark.parametrize("sr", ["maxmin", "addmult", "bool"])
def test_static_engine_matches_library_allocation(oracle, synth, sr):
    """Two calls in a row, the second with a smaller graph: each static
    engine equals a plain engine on the same facts and the oracle; the first
    static engine gives the array up when the second is created."""
    first = None
    for n, m, seed in ((800, 3200, 1), (300, 1200, 2)):
        src, dst, p = synth.er_graph(seed, n, m, weights=True)
        plain = tc_engine(synth, src, dst, p, sr, static=False)
        stat = tc_engine(synth, src, dst, p, sr, static=True)
        got = stat.read("path")
        same(got, plain.read("path"), sr)
        check_closure(got, tc_closure(oracle, n, src, dst, p, sr), sr, f"static {sr} n={n}")
        st = stat.stats()
        assert st["device_allocs"] == 0
        assert 0 < st["workspace_peak"] <= STATIC_BYTES
        stat.run()  # a second run on the same engine
        same(stat.read("path"), plain.read("path"), sr)
        if first is not None:
            from paper_2503_21937_amd import dlfix
            with pytest.raises(dlfix.DLError) as ex:
                first.read("path")
            assert ex.value.status == STATE
        first = stat


def test_static_engine_rejects_too_large_and_workspace(synth):
    from paper_2503_21937_amd import dlfix
    src, dst, p = synth.er_graph(1, 5000, 20000, weights=True)
    e = dlfix.Engine(synth.TC_PROGRAM, "maxmin", static=True)
    e.add_facts("edge", [src, dst], p)
    with pytest.raises(dlfix.DLError) as ex:
        e.run()
    assert ex.value.status == NOMEM
    assert "static workspace" in str(ex.value)
    with pytest.raises(dlfix.DLError) as ex:
        e.set_workspace(1 << 20)
    assert ex.value.status == STATE
    # a smaller input on a new static engine still runs after the failure
    src, dst, p = synth.er_graph(3, 200, 800, weights=True)
    small = tc_engine(synth, src, dst, p, "minplus", static=True)
    plain = tc_engine(synth, src, dst, p, "minplus", static=False)
    np.testing.assert_array_equal(small.read("path")["cols"], plain.read("path")["cols"])
