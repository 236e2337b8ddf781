"""Python binding of libdlfix.so (the HIP fixpoint engine).

Argument marshalling only: every step of the fixpoint runs in the library's
HIP kernels.  Inputs may be numpy arrays (host) or torch tensors (device:
their data pointers are passed and torch's current stream is used).  There is
no fallback: if the library is missing or fails to load, this module raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libdlfix.so")

SEMIRINGS = {"bool": 0, "maxmin": 1, "minplus": 2, "addmult": 3,
             "diff_addmult": 4, "topk": 5, "diff_topk": 6, "diff_maxmin": 7}
STATUS = {0: "OK", 1: "ERR_ARG", 2: "ERR_PARSE", 3: "ERR_UNSUPPORTED", 4: "ERR_STATE",
          5: "ERR_NOMEM", 6: "ERR_CAPACITY", 7: "ERR_PROOF_OVERFLOW", 8: "ERR_HIP"}
EXPORTS = ["dl_load_program", "dl_load_program_static", "dl_clear_facts", "dl_add_facts", "dl_run_fixpoint", "dl_set_workspace",
           "dl_relation_size", "dl_read_relation", "dl_lookup", "dl_backward_rows", "dl_backward", "dl_read_grad",
           "dl_zero_grad", "dl_get_stats", "dl_autotune", "dl_profile", "dl_get_kernel_timing", "dl_get_round_log",
           "dl_last_error", "dl_free"]
KERNEL_FAMILIES = ["join_count", "join_expand", "sort_hist", "sort_scatter", "scan", "reduce",
                   "diff", "merge", "compact", "index", "backward"]


class DLError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Options(C.Structure):
    _fields_ = [("semiring", C.c_int), ("k", C.c_int), ("batched", C.c_int),
                ("stream", C.c_void_p), ("dedup", C.c_int), ("no_graphs", C.c_int), ("no_fused", C.c_int),
                ("lineage", C.c_int), ("lineage_budget", C.c_size_t),
                ("workspace", C.c_void_p), ("workspace_bytes", C.c_size_t),
                ("max_join_outputs", C.c_uint64), ("exact_growth", C.c_int)]


class RelationOut(C.Structure):
    _fields_ = [("sample_ids", C.c_void_p), ("columns", C.c_void_p * 4), ("tags", C.c_void_p),
                ("topk_count", C.c_void_p), ("topk_bits", C.c_void_p), ("topk_prob", C.c_void_p),
                ("fact_ids", C.c_void_p)]


class KernelStats(C.Structure):
    _fields_ = [("launches", C.c_uint64), ("ms", C.c_double), ("bytes", C.c_double)]


class Stats(C.Structure):
    _fields_ = [("strata", C.c_int), ("rounds", C.c_int), ("max_rounds", C.c_int),
                ("candidates", C.c_uint64), ("unique", C.c_uint64), ("derived", C.c_uint64),
                ("lineage", C.c_uint64), ("run_ms", C.c_double), ("device_bytes", C.c_uint64),
                ("key_bits", C.c_uint32), ("id_bits", C.c_uint32), ("sample_bits", C.c_uint32),
                ("dedup", C.c_int), ("orient", C.c_int), ("items", C.c_int), ("tuned_ms", C.c_double),
                ("lineage_mode", C.c_int), ("rows", C.c_int),
                ("device_allocs", C.c_uint64), ("workspace_peak", C.c_uint64), ("index", C.c_int),
                ("topk_words", C.c_int)]


_lib = None


def lib():
    """Load libdlfix.so (built in-tree by build.py); raise if it is missing."""
    global _lib
    if _lib is None:
        # Load torch first so that the library binds to the HIP runtime torch
        # already mapped (one runtime per process: device pointers and streams
        # are then shared, and a second runtime would not see the device).
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(LIB):
            raise ImportError(f"{LIB} is missing: build it with paper_2503_21937_amd/build.py")
        L = C.CDLL(LIB)
        vp, sz = C.c_void_p, C.c_size_t
        L.dl_load_program.argtypes = [C.c_char_p, C.POINTER(Options), C.POINTER(vp)]
        L.dl_load_program_static.argtypes = [C.c_char_p, C.POINTER(Options), C.POINTER(vp)]
        L.dl_clear_facts.argtypes = [vp]
        L.dl_add_facts.argtypes = [vp, C.c_char_p, sz, vp, vp, vp, C.c_int]
        L.dl_run_fixpoint.argtypes = [vp]
        L.dl_set_workspace.argtypes = [vp, vp, sz]
        L.dl_relation_size.argtypes = [vp, C.c_char_p, C.POINTER(sz)]
        L.dl_read_relation.argtypes = [vp, C.c_char_p, sz, C.POINTER(RelationOut), C.c_int,
                                       C.POINTER(sz)]
        L.dl_backward.argtypes = [vp, C.c_char_p, vp, C.c_int]
        L.dl_lookup.argtypes = [vp, C.c_char_p, sz, vp, vp, vp, vp, C.c_int]
        L.dl_backward_rows.argtypes = [vp, C.c_char_p, sz, vp, vp, C.c_int]
        L.dl_read_grad.argtypes = [vp, C.c_char_p, vp, C.c_int]
        L.dl_zero_grad.argtypes = [vp]
        L.dl_get_stats.argtypes = [vp, C.POINTER(Stats)]
        L.dl_autotune.argtypes = [vp, C.c_int, C.c_char_p]
        L.dl_profile.argtypes = [vp, C.c_uint32]
        L.dl_get_kernel_timing.argtypes = [vp, C.c_int, C.POINTER(KernelStats)]
        L.dl_get_round_log.argtypes = [vp, sz, vp, vp, vp, C.POINTER(sz)]
        L.dl_last_error.argtypes = [vp]
        L.dl_last_error.restype = C.c_char_p
        L.dl_free.argtypes = [vp]
        for f in EXPORTS[:-2]:  # all but dl_last_error, dl_free
            getattr(L, f).restype = C.c_int
        _lib = L
    return _lib


def _is_torch(x) -> bool:
    return type(x).__module__.startswith("torch")


def _ptr(x, dtype):
    """(pointer, keepalive, on_device) for a numpy array or torch tensor."""
    if x is None:
        return None, None, None
    if _is_torch(x):
        if not x.is_contiguous():
            x = x.contiguous()
        return x.data_ptr(), x, bool(x.is_cuda)
    a = np.ascontiguousarray(np.asarray(x, dtype=dtype))
    return a.ctypes.data, a, False


def _current_stream() -> int | None:
    try:
        import torch
        if torch.cuda.is_available():
            return torch.cuda.current_stream().cuda_stream
    except Exception:  # torch absent: the engine makes its own stream
        pass
    return None


def _workspace(ws):
    """A device tensor for a workspace argument (None, byte count or tensor)."""
    if ws is None:
        return None
    if isinstance(ws, int):
        import torch
        return torch.empty(ws, dtype=torch.uint8, device="cuda")
    if not (_is_torch(ws) and ws.is_cuda and ws.is_contiguous()):
        raise ValueError("workspace must be a byte count or a contiguous device tensor")
    return ws


class Engine:
    """One fixpoint engine: a program under one semiring (dlfix.h)."""

    DEDUP = {"auto": 0, "sort": 1, "dense": 2, "hash": 3}
    LINEAGE = {"auto": 0, "store": 1, "recompute": 2}

    def __init__(self, program: str, semiring: str = "bool", k: int = 3,
                 batched: bool = False, stream: int | None = None, use_torch_stream: bool = True,
                 dedup: str = "auto", graphs: bool = True, lineage: str = "auto",
                 lineage_budget: int = 0, workspace=None, static: bool = False, fused: bool = True,
                 max_join_outputs: int = 0, exact_growth: bool = False):
        """workspace: None (the library allocates), a byte count (a torch
        uint8 tensor of that size is allocated here and kept), or a device
        tensor whose storage the engine keeps all its buffers in.
        static: keep every buffer in the library's static per-device array
        (dl_load_program_static); no workspace then."""
        self.arity = {}
        for line in program.splitlines():
            line = line.strip()
            if line.startswith(".input") or line.startswith(".output"):
                name, ar = line.split()[1].split("/")
                self.arity[name] = int(ar)
            elif ":-" in line:  # a rule head names a derived relation
                name, args = line.split(":-")[0].split("(", 1)
                args = args.rsplit(")", 1)[0]
                self.arity.setdefault(name.strip(), args.count(",") + 1 if args.strip() else 0)
        self.semiring = semiring
        self.k = k
        self.batched = batched
        if stream is None and use_torch_stream:
            stream = _current_stream()
        self.workspace = _workspace(workspace)
        wp, wn = (None, 0) if self.workspace is None else (self.workspace.data_ptr(), self.workspace.nbytes)
        opts = Options(SEMIRINGS[semiring], k, int(batched), stream, self.DEDUP[dedup], int(not graphs),
                       int(not fused), self.LINEAGE[lineage], lineage_budget, wp, wn, max_join_outputs,
                       int(exact_growth))
        h = C.c_void_p()
        load = lib().dl_load_program_static if static else lib().dl_load_program
        rc = load(program.encode(), C.byref(opts), C.byref(h))
        if rc:
            raise DLError(rc, lib().dl_last_error(None).decode())
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            if _lib is not None:  # at interpreter exit the module may be torn down first
                _lib.dl_free(self.h)
            self.h = None
        self.workspace = None  # only after the engine is gone

    def __del__(self):
        self.close()

    def _check(self, rc):
        if rc:
            raise DLError(rc, lib().dl_last_error(self.h).decode())

    def add_facts(self, rel: str, cols, tags=None, sample=None):
        keep = []
        ptrs = (C.c_void_p * 4)()
        dev = None
        n = None
        for i, c in enumerate(cols):
            p, a, d = _ptr(c, np.uint32)
            keep.append(a)
            ptrs[i] = p
            dev = d if dev is None else dev
            n = int(a.shape[0]) if n is None else n
        tp, ta, _ = _ptr(tags, np.float32)
        sp, sa, _ = _ptr(sample, np.uint32)
        keep += [ta, sa]
        self._check(lib().dl_add_facts(self.h, rel.encode(), n, sp, ptrs, tp, int(bool(dev))))

    def set_workspace(self, workspace):
        """Move the engine's buffers into a new workspace (bytes or tensor;
        None: library allocations).  The previous one is released after."""
        ws = _workspace(workspace)
        wp, wn = (None, 0) if ws is None else (ws.data_ptr(), ws.nbytes)
        self._check(lib().dl_set_workspace(self.h, wp, wn))
        self.workspace = ws

    def clear_facts(self):
        self._check(lib().dl_clear_facts(self.h))

    def run(self):
        self._check(lib().dl_run_fixpoint(self.h))
        return self

    def size(self, rel: str) -> int:
        n = C.c_size_t()
        self._check(lib().dl_relation_size(self.h, rel.encode(), C.byref(n)))
        return n.value

    def read(self, rel: str, device: bool = False) -> dict:
        """Relation in canonical order: dict(sample, cols (n x arity), tags,
        for top-k cnt (n), bits (n x k; n x k x 4 when a sample has more than
        64 probabilistic facts: word w of each proof set), p (n x k), and for differentiable
        max-min fid (n): the number of the input fact each tag comes from)."""
        n = self.size(rel)
        ar = self.arity[rel]
        topk = self.semiring in ("topk", "diff_topk")
        if device:
            import torch
            dv = torch.device("cuda")
            mk = lambda shape, dt: torch.zeros(shape, dtype=dt, device=dv)
            u32, f32, u8, u64 = torch.int32, torch.float32, torch.uint8, torch.int64
        else:
            mk = lambda shape, dt: np.zeros(shape, dt)
            u32, f32, u8, u64 = np.uint32, np.float32, np.uint8, np.uint64
        out = dict(sample=mk(n, u32), cols=[mk(n, u32) for _ in range(ar)], tags=mk(n, f32))
        vid = self.semiring == "diff_maxmin"
        words = self.stats()["topk_words"] if topk else 1
        if topk:
            shape = (self.k, n) if words == 1 else (self.k, n, words)
            out.update(cnt=mk(n, u8), bits=mk(shape, u64), p=mk((self.k, n), f32))
        if vid:
            out["fid"] = mk(n, u32)
        ro = RelationOut()
        ptr = (lambda t: t.data_ptr()) if device else (lambda a: a.ctypes.data)
        if n:
            ro.sample_ids = ptr(out["sample"])
            for c in range(ar):
                ro.columns[c] = ptr(out["cols"][c])
            ro.tags = ptr(out["tags"])
            if topk:
                ro.topk_count = ptr(out["cnt"])
                ro.topk_bits = ptr(out["bits"])
                ro.topk_prob = ptr(out["p"])
            if vid:
                ro.fact_ids = ptr(out["fid"])
        w = C.c_size_t()
        self._check(lib().dl_read_relation(self.h, rel.encode(), n, C.byref(ro), int(device),
                                           C.byref(w)))
        if not device:
            out["cols"] = np.stack(out["cols"], 1) if ar else np.zeros((n, 0), np.uint32)
            if topk:
                out["bits"] = (out["bits"].T if words == 1 else out["bits"].transpose(1, 0, 2)).copy()
                out["p"] = out["p"].T.copy()
        return out

    def lookup(self, rel: str, cols, sample=None, device: bool = False):
        """Rows (canonical index or -1) and tags of the given tuples."""
        keep = []
        ptrs = (C.c_void_p * 4)()
        n, dev = None, False
        for i, c in enumerate(cols):
            p_, a, d = _ptr(c, np.uint32)
            keep.append(a)
            ptrs[i] = p_
            n, dev = int(a.shape[0]), bool(d)
        sp, sa, _ = _ptr(sample, np.uint32)
        keep.append(sa)
        if dev:
            import torch
            rows = torch.empty(n, dtype=torch.int64, device=cols[0].device)
            tags = torch.empty(n, dtype=torch.float32, device=cols[0].device)
            rp, tp = rows.data_ptr(), tags.data_ptr()
        else:
            rows = np.empty(n, np.int64)
            tags = np.empty(n, np.float32)
            rp, tp = rows.ctypes.data, tags.ctypes.data
        self._check(lib().dl_lookup(self.h, rel.encode(), n, sp, ptrs, rp, tp, int(dev)))
        return rows, tags

    def backward_rows(self, rel: str, rows, grad):
        rp, ra, dev = _ptr(rows, np.int64)
        gp, ga, _ = _ptr(grad, np.float32)
        n = int(ra.shape[0])
        self._check(lib().dl_backward_rows(self.h, rel.encode(), n, rp, gp, int(bool(dev))))

    def backward(self, rel: str, grad_out):
        p, a, dev = _ptr(grad_out, np.float32)
        self._check(lib().dl_backward(self.h, rel.encode(), p, int(bool(dev))))

    def grad(self, rel: str, n: int, out=None):
        if out is None:
            out = np.zeros(n, np.float32)
        p, a, dev = _ptr(out, np.float32)
        self._check(lib().dl_read_grad(self.h, rel.encode(), p, int(bool(dev))))
        return out

    def zero_grad(self):
        self._check(lib().dl_zero_grad(self.h))

    def autotune(self, trials: int = 3, cache: str | None = None) -> dict:
        """Pick the fastest execution configuration for the current facts."""
        self._check(lib().dl_autotune(self.h, trials, None if cache is None else cache.encode()))
        st = self.stats()
        return {k: st[k] for k in ("dedup", "orient", "items", "rows", "tuned_ms")}

    def profile(self, families=None):
        """Time the given kernel families (names; None = all, [] = off)."""
        if families is None:
            mask = (1 << len(KERNEL_FAMILIES)) - 1
        else:
            mask = 0
            for f in families:
                mask |= 1 << KERNEL_FAMILIES.index(f)
        self._check(lib().dl_profile(self.h, mask))

    def kernel_stats(self) -> dict:
        out = {}
        for i, name in enumerate(KERNEL_FAMILIES):
            ks = KernelStats()
            self._check(lib().dl_get_kernel_timing(self.h, i, C.byref(ks)))
            out[name] = dict(launches=ks.launches, ms=ks.ms, bytes=ks.bytes)
        return out

    ROUND_KINDS = {1: "first", 2: "plain", 3: "fused", 4: "batched"}

    def round_log(self) -> dict:
        """Per-round sizes of the last run: dict(new, derivations (2^64 - 1
        where only the device's total is known), stratum, kind: 1 first
        round, 2 later round, 3 fused-round launch, 4 batched round)."""
        n = C.c_size_t()
        self._check(lib().dl_get_round_log(self.h, 0, None, None, None, C.byref(n)))
        new = np.zeros(n.value, np.uint64)
        der = np.zeros(n.value, np.uint64)
        info = np.zeros(n.value, np.uint32)
        if n.value:
            self._check(lib().dl_get_round_log(self.h, n.value, new.ctypes.data, der.ctypes.data, info.ctypes.data,
                                               C.byref(n)))
        return dict(new=new, derivations=der, stratum=info >> 8, kind=info & 0xff)

    def stats(self) -> dict:
        s = Stats()
        self._check(lib().dl_get_stats(self.h, C.byref(s)))
        return {f: getattr(s, f) for f, _ in Stats._fields_}
