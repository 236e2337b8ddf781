"""ctypes front end of the CPU oracle -- TEST INFRASTRUCTURE ONLY.

Only tests, the smoke check and the benchmark's CPU-baseline leg use this
module.  It loads `oracle/libdlref.so` (built by `build()` with g++ from the
C++ sources beside it) and shares no code with the HIP product path.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libdlref.so")
SOURCES = ["naive.cpp", "special.cpp"]

SEMIRINGS = {"bool": 0, "maxmin": 1, "minplus": 2, "addmult": 3,
             "diff_addmult": 4, "topk": 5, "diff_topk": 6, "diff_maxmin": 7}


def build(force: bool = False) -> str:
    """Compile the oracle with g++ (binary32/64 IEEE, no FP contraction)."""
    srcs = [os.path.join(HERE, s) for s in SOURCES]
    if not force and os.path.exists(LIB) and all(
            os.path.getmtime(LIB) >= os.path.getmtime(s)
            for s in srcs + [os.path.join(HERE, "dlref.h")]):
        return LIB
    tmp = LIB + ".tmp"
    cmd = ["g++", "-std=c++17", "-O2", "-fPIC", "-shared", "-ffp-contract=off",
           "-fno-fast-math", "-Wall", "-o", tmp] + srcs
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = C.CDLL(LIB)
        vp, sz = C.c_void_p, C.c_size_t
        L.ref_create.argtypes = [C.c_char_p, C.c_int, C.c_int, C.c_int,
                                 C.POINTER(vp), C.c_char_p, sz]
        L.ref_add_facts.argtypes = [vp, C.c_char_p, sz, vp, vp, vp]
        L.ref_run.argtypes = [vp]
        L.ref_size.argtypes = [vp, C.c_char_p]
        L.ref_size.restype = C.c_long
        L.ref_rounds.argtypes = [vp, C.c_int]
        L.ref_num_strata.argtypes = [vp]
        L.ref_read.argtypes = [vp, C.c_char_p] + [vp] * 8
        L.ref_backward.argtypes = [vp, C.c_char_p, vp]
        L.ref_read_fid.argtypes = [vp, C.c_char_p, vp]
        L.ref_read_bits.argtypes = [vp, C.c_char_p, vp]
        L.ref_vid_op.argtypes = [C.c_int, C.c_double, C.c_uint32, C.c_double, C.c_uint32,
                                 C.POINTER(C.c_double), C.POINTER(C.c_uint32)]
        L.ref_read_grad.argtypes = [vp, C.c_char_p, vp]
        L.ref_zero_grad.argtypes = [vp]
        L.ref_error.argtypes = [vp]
        L.ref_error.restype = C.c_char_p
        L.ref_free.argtypes = [vp]
        L.ref_scalar_op.argtypes = [C.c_int, C.c_int, C.c_double, C.c_double, C.POINTER(C.c_double)]
        L.ref_scalar_identity.argtypes = [C.c_int, C.c_int, C.POINTER(C.c_double)]
        L.ref_topk_op.argtypes = [C.c_int, C.c_int, C.c_int, vp, C.c_int, vp, vp, vp, vp, vp]
        L.ref_tc_column.argtypes = [C.c_int, sz, vp, vp, vp, C.c_int, C.c_uint32,
                                    vp, vp, vp, vp, vp, vp]
        L.ref_andersen.argtypes = [C.c_uint32, sz, vp, sz, vp, sz, vp, sz, vp]
        L.ref_andersen.restype = vp
        L.ref_pts_size.argtypes = [vp]
        L.ref_pts_size.restype = C.c_long
        L.ref_pts_read.argtypes = [vp, vp, vp]
        L.ref_pts_free.argtypes = [vp]
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


class Oracle:
    """Naive Jacobi evaluation of a program under one semiring."""

    def __init__(self, program: str, semiring: str, k: int = 3, batched: bool = False):
        self.arity = {}
        for line in program.splitlines():
            line = line.strip()
            if line.startswith(".input") or line.startswith(".output"):
                name, ar = line.split()[1].split("/")
                self.arity[name] = int(ar)
            elif ":-" in line:  # a rule head names a derived relation
                head = line.split(":-")[0]
                name, args = head.split("(", 1)
                args = args.rsplit(")", 1)[0]
                self.arity.setdefault(name.strip(), args.count(",") + 1 if args.strip() else 0)
        self.semiring = semiring
        self.batched = batched
        h = C.c_void_p()
        err = C.create_string_buffer(512)
        rc = lib().ref_create(program.encode(), SEMIRINGS[semiring], k, int(batched),
                              C.byref(h), err, 512)
        if rc:
            raise ValueError(err.value.decode())
        self.h = h

    def __del__(self):
        if getattr(self, "h", None):
            lib().ref_free(self.h)
            self.h = None

    def _err(self, what):
        raise RuntimeError(f"{what}: {lib().ref_error(self.h).decode()}")

    def add_facts(self, rel: str, cols, tags=None, sample=None):
        cols = [np.asarray(c, np.uint32) for c in cols]
        n = cols[0].size
        rows = np.ascontiguousarray(np.stack(cols, axis=1).astype(np.uint32))
        t = None if tags is None else np.ascontiguousarray(np.asarray(tags, np.float32))
        s = None if sample is None else np.ascontiguousarray(np.asarray(sample, np.uint32))
        if lib().ref_add_facts(self.h, rel.encode(), n, _p(s), _p(rows), _p(t)):
            self._err("add_facts")

    def run(self):
        lib().ref_run(self.h)
        return self

    def rounds(self, stratum: int = -1) -> int:
        ns = lib().ref_num_strata(self.h)
        return lib().ref_rounds(self.h, ns - 1 if stratum < 0 else stratum)

    def size(self, rel: str) -> int:
        return int(lib().ref_size(self.h, rel.encode()))

    def read(self, rel: str) -> dict:
        n = self.size(rel)
        ar = self.arity.get(rel)
        if ar is None:
            raise KeyError(rel)
        s = np.zeros(n, np.uint32)
        cols = np.zeros((n, ar), np.uint32)
        val = np.zeros(n, np.float64)
        cnt = np.zeros(n, np.int32)
        bits = np.zeros((n, 3), np.uint64)
        p = np.zeros((n, 3), np.float32)
        prob = np.zeros(n, np.float64)
        rf = np.zeros(n, np.int32)
        lib().ref_read(self.h, rel.encode(), _p(s), _p(cols), _p(val), _p(cnt),
                       _p(bits), _p(p), _p(prob), _p(rf))
        wide = np.zeros((n, 3, 4), np.uint64)
        lib().ref_read_bits(self.h, rel.encode(), _p(wide))
        return dict(sample=s, cols=cols, value=val, cnt=cnt, bits=bits, p=p,
                    prob=prob, round=rf, bits_wide=wide)

    def fid(self, rel: str) -> np.ndarray:
        """Differentiable max-min: the input fact number each tuple's tag comes from."""
        out = np.zeros(self.size(rel), np.uint32)
        if lib().ref_read_fid(self.h, rel.encode(), _p(out)):
            self._err("read_fid")
        return out

    def backward(self, out_rel: str, grad_out):
        g = np.ascontiguousarray(np.asarray(grad_out, np.float64))
        if lib().ref_backward(self.h, out_rel.encode(), _p(g)):
            self._err("backward")

    def grad(self, in_rel: str, n: int) -> np.ndarray:
        g = np.zeros(n, np.float64)
        if lib().ref_read_grad(self.h, in_rel.encode(), _p(g)):
            self._err("read_grad")
        return g

    def zero_grad(self):
        lib().ref_zero_grad(self.h)


def vid_op(op: str, a, b):
    """Differentiable max-min pair operation ('plus' or 'times') on (value, fact) pairs."""
    ov, oid = C.c_double(), C.c_uint32()
    lib().ref_vid_op(0 if op == "plus" else 1, float(a[0]), int(a[1]), float(b[0]), int(b[1]), C.byref(ov),
                     C.byref(oid))
    return ov.value, oid.value


def tc_column(n: int, src, dst, w, semiring: str, z: int, grad_col=None):
    """One target column of the transitive-closure fixpoint (see special.cpp).

    Returns dict(present, tag, found, rounds[, grad_edge])."""
    src = np.ascontiguousarray(src, np.uint32)
    dst = np.ascontiguousarray(dst, np.uint32)
    w = np.ascontiguousarray(np.ones(src.size, np.float32) if w is None else w, np.float32)
    pres = np.zeros(n, np.uint8)
    tag = np.zeros(n, np.float64)
    found = np.zeros(n, np.int32)
    rounds = np.zeros(1, np.int32)
    gc = ge = None
    if grad_col is not None:
        gc = np.ascontiguousarray(grad_col, np.float64)
        ge = np.zeros(src.size, np.float64)
    rc = lib().ref_tc_column(n, src.size, _p(src), _p(dst), _p(w), SEMIRINGS[semiring], z,
                             _p(pres), _p(tag), _p(found), _p(rounds), _p(gc), _p(ge))
    if rc:
        raise ValueError(f"ref_tc_column failed ({rc})")
    out = dict(present=pres.astype(bool), tag=tag, found=found, rounds=int(rounds[0]))
    if ge is not None:
        out["grad_edge"] = ge
    return out


def andersen(nvars: int, rels: dict) -> tuple[np.ndarray, np.ndarray]:
    """Least points-to solution by worklist propagation; (v, o) sorted."""
    def rows(name):
        a, b = rels[name]
        return np.ascontiguousarray(np.stack([a, b], 1).astype(np.uint32))
    A, S, L, T = rows("addr"), rows("assign"), rows("load"), rows("store")
    h = lib().ref_andersen(nvars, A.shape[0], _p(A), S.shape[0], _p(S), L.shape[0], _p(L),
                           T.shape[0], _p(T))
    n = lib().ref_pts_size(h)
    v = np.zeros(n, np.uint32)
    o = np.zeros(n, np.uint32)
    lib().ref_pts_read(h, _p(v), _p(o))
    lib().ref_pts_free(h)
    return v, o


def scalar_op(semiring: str, op: str, a: float, b: float) -> float:
    out = C.c_double()
    if lib().ref_scalar_op(SEMIRINGS[semiring], 1 if op == "times" else 0, a, b, C.byref(out)):
        raise ValueError(semiring)
    return out.value


def scalar_identity(semiring: str, which: str) -> float:
    out = C.c_double()
    if lib().ref_scalar_identity(SEMIRINGS[semiring], 1 if which == "one" else 0, C.byref(out)):
        raise ValueError(semiring)
    return out.value


def topk_op(k: int, op: str, a, b, q):
    """a, b: lists of proof bitsets; returns (bits list, probs list)."""
    ab = np.zeros(3, np.uint64)
    bb = np.zeros(3, np.uint64)
    ab[: len(a)] = a
    bb[: len(b)] = b
    qa = np.ascontiguousarray(q, np.float32)
    cnt = C.c_int()
    ob = np.zeros(3, np.uint64)
    op_ = np.zeros(3, np.float32)
    if lib().ref_topk_op(k, 1 if op == "times" else 0, len(a), _p(ab), len(b), _p(bb), _p(qa), C.byref(cnt),
                         _p(ob), _p(op_)):
        raise ValueError("topk_op")
    return [int(x) for x in ob[: cnt.value]], [float(x) for x in op_[: cnt.value]]
