"""CPU checks of the C-ABI library: it loads, exports every function that
include/dlfix.h declares, and rejects bad programs before touching a GPU."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def dl():
    from paper_2503_21937_amd import dlfix
    if not os.path.exists(dlfix.LIB):
        from paper_2503_21937_amd import build
        build.build()
    return dlfix


def declared():
    text = open(os.path.join(ROOT, "include", "dlfix.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dl_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared()
    for n in ["dl_load_program", "dl_add_facts", "dl_run_fixpoint", "dl_read_relation",
              "dl_backward", "dl_read_grad", "dl_free"]:
        assert n in names


def test_library_exports_every_declared_symbol(dl):
    lib = C.CDLL(dl.LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(dl.EXPORTS) == declared()


@pytest.mark.parametrize("text,status", [
    ("path(x, y) :- edge(x, y", 2),                               # parse error
    ("path(x, z) :- edge(x, 3).", 3),                             # unbound head variable (beside a constant)
    ("path(x, w) :- edge(x, y).", 3),                             # unbound head variable
    ("p(x) :- e(x, y), z > 1.", 3),                               # condition on an unbound variable
    ("p(x, w + 1) :- e(x, y).", 3),                               # head expression on an unbound variable
    ("p(x) :- x > 1.", 3),                                        # no body atom
    ("p(x) :- e(x, y), x <> y.", 2),                              # unknown comparison
    ("p(a) :- q(a), r(b).", 3),                                   # disconnected body
    ("p(a) :- q(a, b), r(b, c), s(c, d), t(d, a).", 3),           # four atoms
    (".input edge/2\nedge(x, y) :- edge(y, x).", 3),              # head on an input
])
def test_rejected_programs(dl, text, status):
    with pytest.raises(dl.DLError) as ex:
        dl.Engine(text, "bool", use_torch_stream=False)
    assert ex.value.status == status


def test_frozen_semiring_accepts_nonlinear_recursion(dl):
    # several atoms of the rule's own stratum: each is planned as the delta
    # atom once, with the atoms before it on the stable part (Appendix A)
    # without a device the load gets past parsing and planning and only then
    # fails on stream creation (DL_ERR_HIP)
    def loads(text, sr):
        try:
            dl.Engine(text, sr, use_torch_stream=False)
        except dl.DLError as ex:
            assert ex.status == 8, ex
    prog = ".input e/2\np(x, y) :- e(x, y).\np(x, z) :- p(x, y), p(y, z)."
    for sr in ("addmult", "diff_addmult"):
        loads(prog, sr)
    prog3 = ".input e/2\np(x, y) :- e(x, y).\np(x, w) :- p(x, y), p(y, z), p(z, w)."
    loads(prog3, "addmult")
    with pytest.raises(dl.DLError) as ex:
        dl.Engine(prog3, "diff_addmult", use_torch_stream=False)
    assert ex.value.status == 3


def test_expressions_are_accepted(dl):
    """Constants and repeated variables in atoms, comparisons, arithmetic head
    terms and nullary heads get past parsing and planning (without a device
    the load then fails on stream creation, DL_ERR_HIP)."""
    for text in ("path(x, z) :- edge(x, 3), edge(3, z).",
                 "loop(x) :- edge(x, x).",
                 "sg(x, y) :- edge(p, x), edge(p, y), x != y.",
                 "walk(x, z, d + 1) :- walk(x, y, d), edge(y, z), d < 4.",
                 "q(x, (y * 3 + 1) % 7, y / 2) :- e(x, y), x <= y, x >= 1, y == 2 * x.",
                 "any() :- e(x, y), x != y."):
        with pytest.raises(dl.DLError) as ex:
            dl.Engine(".input edge/2\n.input e/2\n" + text, "bool", use_torch_stream=False)
        assert ex.value.status == 8, (text, ex.value)


def test_bad_options(dl):
    with pytest.raises(dl.DLError) as ex:
        dl.Engine(".input e/2\np(x,y) :- e(x,y).", "topk", k=4, use_torch_stream=False)
    assert ex.value.status == 1
