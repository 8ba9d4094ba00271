"""Python binding of the C-ABI library ``libcbc.so`` (argument marshalling only).

Every step of the compression runs in the library's HIP kernels; this module only packs host
arrays, passes torch device pointers and the current HIP stream, and raises on error codes.
PyTorch provides device memory and streams. The library must be built (``build_lib.py``); there is
no fallback path: importing without the library, or calling without a GPU, raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcbc.so")

FP64, MIXED = 0, 1
PRECISIONS = {"fp64": FP64, "mixed": MIXED}
METHODS = {"cbc": 0, "naive": 1, "src": 2, "dm": 3, "zipup": 4}


class CbcError(RuntimeError):
    pass


class _Tree(ctypes.Structure):
    _fields_ = [("n_nodes", ctypes.c_int32), ("parent", ctypes.POINTER(ctypes.c_int32)),
                ("phys", ctypes.POINTER(ctypes.c_int32)), ("chi", ctypes.POINTER(ctypes.c_int32)),
                ("dop", ctypes.POINTER(ctypes.c_int32))]


class _Tensors(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("offset", ctypes.POINTER(ctypes.c_int64))]


class _Out(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("offset", ctypes.POINTER(ctypes.c_int64)),
                ("bond", ctypes.POINTER(ctypes.c_int32))]


NCLASS = 6
CLASSES = ("contract", "gram", "qrmul", "eig", "chol", "other")


class PlanSummary(ctypes.Structure):
    _fields_ = [("persistent_bytes", ctypes.c_size_t), ("scratch_bytes", ctypes.c_size_t),
                ("table_bytes", ctypes.c_size_t), ("launches", ctypes.c_int32 * NCLASS),
                ("flops", ctypes.c_double * NCLASS)]


class Stats(ctypes.Structure):
    _fields_ = [("profile", ctypes.c_int32), ("n_kernels", ctypes.c_int32),
                ("n_eig", ctypes.c_int32), ("max_eig_dim", ctypes.c_int32),
                ("graph_replayed", ctypes.c_int32), ("launches", ctypes.c_int32 * NCLASS),
                ("flops", ctypes.c_double * NCLASS), ("bytes", ctypes.c_double * NCLASS),
                ("ms", ctypes.c_double * NCLASS)]

    def as_dict(self):
        return {c: dict(launches=int(self.launches[k]), flops=float(self.flops[k]),
                        bytes=float(self.bytes[k]), ms=float(self.ms[k]))
                for k, c in enumerate(CLASSES)}


class TruncRecord(ctypes.Structure):
    _fields_ = [("node", ctypes.c_int32), ("sweep", ctypes.c_int32), ("dim", ctypes.c_int32),
                ("kmax", ctypes.c_int32), ("kept", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("discarded", ctypes.c_double), ("gap", ctypes.c_double)]


class Report(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("dropped_pivots", ctypes.c_int32),
                ("n_trunc", ctypes.c_int32), ("capacity", ctypes.c_int32),
                ("trunc", ctypes.POINTER(TruncRecord))]


STATUS = {0: "ok", -1: "einval", -2: "eshape", -3: "enomem", -4: "ehip", -5: "enotpd",
          -6: "eunsup", -7: "enotbuilt", -8: "etimeout"}

_lib = None


def lib():
    """Load libcbc.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise CbcError(f"{LIB_PATH} is missing: build it with paper_2601_19650_amd/build_lib.py")
        L = ctypes.CDLL(LIB_PATH)
        L.cbc_create.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
        L.cbc_create.restype = ctypes.c_int
        L.cbc_destroy.argtypes = [ctypes.c_void_p]
        L.cbc_destroy.restype = None
        L.cbc_status_str.argtypes = [ctypes.c_int]
        L.cbc_status_str.restype = ctypes.c_char_p
        L.cbc_query.argtypes = [ctypes.c_void_p, ctypes.POINTER(_Tree), ctypes.c_int32, ctypes.c_int,
                                ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t),
                                ctypes.POINTER(ctypes.c_int64)]
        L.cbc_query.restype = ctypes.c_int
        L.cbc_plan_bonds.argtypes = [ctypes.c_void_p, ctypes.POINTER(_Tree), ctypes.c_int32,
                                     ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]
        L.cbc_plan_bonds.restype = ctypes.c_int
        L.cbc_plan_info.argtypes = [ctypes.c_void_p, ctypes.POINTER(_Tree), ctypes.c_int32,
                                    ctypes.c_int, ctypes.c_int32, ctypes.c_int32,
                                    ctypes.POINTER(PlanSummary)]
        L.cbc_plan_info.restype = ctypes.c_int
        for name in ("cbc_apply", "cbc_apply_naive"):
            f = getattr(L, name)
            f.argtypes = [ctypes.c_void_p, ctypes.POINTER(_Tensors), ctypes.POINTER(_Tensors),
                          ctypes.POINTER(_Tree), ctypes.c_int32, ctypes.c_double, ctypes.c_int,
                          ctypes.c_void_p, ctypes.c_size_t, ctypes.POINTER(_Out), ctypes.c_void_p,
                          ctypes.POINTER(Stats)]
            f.restype = ctypes.c_int
        L.cbc_apply_batched.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(_Tensors),
                                        ctypes.POINTER(_Tensors), ctypes.POINTER(_Tree),
                                        ctypes.c_int32, ctypes.c_double, ctypes.c_int,
                                        ctypes.c_void_p, ctypes.c_size_t, ctypes.POINTER(_Out),
                                        ctypes.c_void_p, ctypes.POINTER(Stats)]
        L.cbc_apply_batched.restype = ctypes.c_int
        L.cbc_apply_noalloc.argtypes = [ctypes.c_void_p, ctypes.POINTER(_Tensors),
                                        ctypes.POINTER(_Tensors), ctypes.POINTER(_Tree),
                                        ctypes.c_int32, ctypes.c_double, ctypes.c_int,
                                        ctypes.POINTER(_Out), ctypes.c_void_p, ctypes.POINTER(Stats)]
        L.cbc_apply_noalloc.restype = ctypes.c_int
        L.cbc_apply_split.argtypes = [ctypes.c_void_p, ctypes.POINTER(_Tensors),
                                      ctypes.POINTER(_Tensors), ctypes.POINTER(_Tree),
                                      ctypes.c_int32, ctypes.c_double, ctypes.c_int,
                                      ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p,
                                      ctypes.c_size_t, ctypes.POINTER(_Out), ctypes.c_void_p,
                                      ctypes.POINTER(Stats)]
        L.cbc_apply_split.restype = ctypes.c_int
        L.cbc_apply_src.argtypes = [ctypes.c_void_p, ctypes.POINTER(_Tensors),
                                    ctypes.POINTER(_Tensors), ctypes.POINTER(_Tensors),
                                    ctypes.POINTER(_Tree), ctypes.c_int32, ctypes.c_int,
                                    ctypes.c_void_p, ctypes.c_size_t, ctypes.POINTER(_Out),
                                    ctypes.c_void_p, ctypes.POINTER(Stats)]
        L.cbc_apply_src.restype = ctypes.c_int
        L.cbc_apply_many.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(CProblem),
                                     ctypes.c_int, ctypes.c_int32, ctypes.POINTER(ctypes.c_void_p),
                                     ctypes.POINTER(ctypes.c_size_t), ctypes.c_void_p]
        L.cbc_apply_many.restype = ctypes.c_int
        L.cbc_apply_dm.argtypes = [ctypes.c_void_p, ctypes.POINTER(_Tensors),
                                   ctypes.POINTER(_Tensors), ctypes.POINTER(_Tree), ctypes.c_int32,
                                   ctypes.c_int, ctypes.c_void_p, ctypes.c_size_t,
                                   ctypes.POINTER(_Out), ctypes.c_void_p, ctypes.POINTER(Stats)]
        L.cbc_apply_dm.restype = ctypes.c_int
        L.cbc_apply_zipup.argtypes = L.cbc_apply_dm.argtypes
        L.cbc_apply_zipup.restype = ctypes.c_int
        L.cbc_autotune.argtypes = [ctypes.c_void_p, ctypes.c_char_p]
        L.cbc_autotune.restype = ctypes.c_int
        L.cbc_read_report.argtypes = [ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32,
                                      ctypes.c_void_p, ctypes.POINTER(Report)]
        L.cbc_read_report.restype = ctypes.c_int
        _lib = L
    return _lib


EXPORTED = ("cbc_create", "cbc_destroy", "cbc_status_str", "cbc_query", "cbc_plan_bonds",
            "cbc_apply", "cbc_apply_batched", "cbc_apply_naive", "cbc_autotune", "cbc_read_report",
            "cbc_apply_noalloc", "cbc_plan_info", "cbc_apply_split", "cbc_apply_src",
            "cbc_apply_many", "cbc_apply_dm", "cbc_apply_zipup")


def _check(code, what):
    if code != 0:
        msg = lib().cbc_status_str(code).decode()
        raise CbcError(f"{what} failed with status {code}: {msg}")


def _i32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32))


class Context:
    """Owns a library context (plan cache)."""

    def __init__(self):
        h = ctypes.c_void_p()
        _check(lib().cbc_create(ctypes.byref(h)), "cbc_create")
        self.h = h

    def autotune(self, cache_path=None):
        """Tune the contractions of plans built from now on (see cbc_autotune); cache_path: text
        file of earlier choices, read now and appended to."""
        path = None if cache_path is None else str(cache_path).encode()
        _check(lib().cbc_autotune(self.h, path), "cbc_autotune")
        return self

    def close(self):
        if self.h:
            lib().cbc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Tree:
    """Host description of the tree and its bond dimensions (kept alive for ctypes)."""

    def __init__(self, parent, phys, chi, dop):
        self.parent, self.phys, self.chi, self.dop = (_i32(parent), _i32(phys), _i32(chi), _i32(dop))
        self.n = len(self.parent)
        P = ctypes.POINTER(ctypes.c_int32)
        self.c = _Tree(self.n, self.parent.ctypes.data_as(P), self.phys.ctypes.data_as(P),
                       self.chi.ctypes.data_as(P), self.dop.ctypes.data_as(P))
        self.children = [[j for j in range(self.n) if self.parent[j] == i] for i in range(self.n)]

    def state_shape(self, i):
        return (int(self.phys[i]), int(self.chi[i])) + tuple(int(self.chi[c]) for c in self.children[i])

    def op_shape(self, i):
        d = int(self.phys[i])
        return (d, d, int(self.dop[i])) + tuple(int(self.dop[c]) for c in self.children[i])

    @staticmethod
    def of(problem):
        return Tree(problem.parent, problem.phys, problem.chi, problem.dop)


def pack(tensors, device):
    """Pack node tensors (numpy complex128) into one device buffer; returns (buffer, offsets)."""
    return pack_batch([tensors], device)


def pack_batch(networks, device):
    """Pack several networks of the same shape back to back (instance b at b * total elements)."""
    import torch
    sizes = [int(np.prod(t.shape)) for t in networks[0]]
    off = np.zeros(len(sizes), dtype=np.int64)
    off[1:] = np.cumsum(sizes)[:-1]
    flat = np.concatenate([np.ascontiguousarray(t, dtype=np.complex128).reshape(-1)
                           for net in networks for t in net])
    return torch.from_numpy(flat).to(device), off


class Compressor:
    """One problem shape: queries sizes once, owns workspace and output buffers, and runs the
    compression (``method`` "cbc", "naive", "src", "dm" or "zipup", ``precision`` "fp64" or "mixed"; "src"
    takes its sketch matrices as run()'s ``sketch`` = (device buffer, offsets) from pack())."""

    def __init__(self, ctx, tree, max_bond, precision="fp64", method="cbc", device="cuda", batch=1,
                 scratch=None):
        """`scratch`: a device byte tensor shared with other Compressors whose calls are ordered
        with this one's (same stream); the workspace then holds only the part that lives through
        a call, and run() goes through cbc_apply_split (single instances of the CBC method)."""
        import torch
        self.ctx, self.tree, self.max_bond = ctx, tree, int(max_bond)
        self.batch = int(batch)
        self.prec = PRECISIONS[precision]
        self.method = METHODS[method]
        ws = ctypes.c_size_t()
        self.out_off = np.zeros(tree.n + 1, dtype=np.int64)
        _check(lib().cbc_query(ctx.h, ctypes.byref(tree.c), self.max_bond, self.prec, self.method,
                               ctypes.byref(ws), self.out_off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))),
               "cbc_query")
        self.scratch = scratch
        if scratch is not None:
            if self.batch != 1 or self.method != 0:
                raise ValueError("a shared scratch serves single CBC calls only")
            need = scratch_need(ctx, tree, self.max_bond, precision)
            if scratch.numel() < need["scratch_bytes"]:
                raise ValueError("shared scratch smaller than this problem needs")
            self.ws_bytes = need["persistent_bytes"]
        else:
            self.ws_bytes = int(ws.value) * self.batch
        self.workspace = torch.empty(max(self.ws_bytes, 256), dtype=torch.uint8, device=device)
        self.out = torch.zeros(int(self.out_off[-1]) * self.batch, dtype=torch.complex128,
                               device=device)
        self.bond = np.zeros(tree.n, dtype=np.int32)
        self.stats = Stats()

    def run(self, op_buf, op_off, st_buf, st_off, tol=0.0, stream=None, profile=False, sketch=None):
        import torch
        self.stats.profile = int(bool(profile))
        op_off = np.ascontiguousarray(op_off, dtype=np.int64)
        st_off = np.ascontiguousarray(st_off, dtype=np.int64)
        I64 = ctypes.POINTER(ctypes.c_int64)
        ttno = _Tensors(op_buf.data_ptr(), op_off.ctypes.data_as(I64))
        ttns = _Tensors(st_buf.data_ptr(), st_off.ctypes.data_as(I64))
        out = _Out(self.out.data_ptr(), self.out_off.ctypes.data_as(I64),
                   self.bond.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        if self.batch > 1:
            _check(lib().cbc_apply_batched(self.ctx.h, self.batch, ctypes.byref(ttno), ctypes.byref(ttns),
                                           ctypes.byref(self.tree.c), self.max_bond, float(tol),
                                           self.prec, self.workspace.data_ptr(), self.ws_bytes,
                                           ctypes.byref(out), ctypes.c_void_p(stream),
                                           ctypes.byref(self.stats)), "cbc_apply_batched")
            return self.out, self.bond
        if self.method == 2:
            if sketch is None:
                raise ValueError("the randomised method needs its sketch matrices")
            sk_off = np.ascontiguousarray(sketch[1], dtype=np.int64)
            sk = _Tensors(sketch[0].data_ptr(), sk_off.ctypes.data_as(I64))
            _check(lib().cbc_apply_src(self.ctx.h, ctypes.byref(ttno), ctypes.byref(ttns),
                                       ctypes.byref(sk), ctypes.byref(self.tree.c), self.max_bond,
                                       self.prec, self.workspace.data_ptr(), self.ws_bytes,
                                       ctypes.byref(out), ctypes.c_void_p(stream),
                                       ctypes.byref(self.stats)), "cbc_apply_src")
            return self.out, self.bond
        if self.scratch is not None:
            _check(lib().cbc_apply_split(self.ctx.h, ctypes.byref(ttno), ctypes.byref(ttns),
                                         ctypes.byref(self.tree.c), self.max_bond, float(tol),
                                         self.prec, self.workspace.data_ptr(), self.ws_bytes,
                                         self.scratch.data_ptr(), self.scratch.numel(),
                                         ctypes.byref(out), ctypes.c_void_p(stream),
                                         ctypes.byref(self.stats)), "cbc_apply_split")
            return self.out, self.bond
        if self.method in (3, 4):
            name = "cbc_apply_dm" if self.method == 3 else "cbc_apply_zipup"
            _check(getattr(lib(), name)(self.ctx.h, ctypes.byref(ttno), ctypes.byref(ttns),
                                        ctypes.byref(self.tree.c), self.max_bond, self.prec,
                                        self.workspace.data_ptr(), self.ws_bytes,
                                        ctypes.byref(out), ctypes.c_void_p(stream),
                                        ctypes.byref(self.stats)), name)
            return self.out, self.bond
        fn = lib().cbc_apply if self.method == 0 else lib().cbc_apply_naive
        _check(fn(self.ctx.h, ctypes.byref(ttno), ctypes.byref(ttns), ctypes.byref(self.tree.c),
                  self.max_bond, float(tol), self.prec, self.workspace.data_ptr(), self.ws_bytes,
                  ctypes.byref(out), ctypes.c_void_p(stream), ctypes.byref(self.stats)),
               "cbc_apply" if self.method == 0 else "cbc_apply_naive")
        return self.out, self.bond

    def run_noalloc(self, op_buf, op_off, st_buf, st_off, tol=0.0, stream=None):
        """The same compression through cbc_apply_noalloc (the library's static per-GPU scratch
        instead of this object's workspace); results go to self.out as with run()."""
        import torch
        op_off = np.ascontiguousarray(op_off, dtype=np.int64)
        st_off = np.ascontiguousarray(st_off, dtype=np.int64)
        I64 = ctypes.POINTER(ctypes.c_int64)
        ttno = _Tensors(op_buf.data_ptr(), op_off.ctypes.data_as(I64))
        ttns = _Tensors(st_buf.data_ptr(), st_off.ctypes.data_as(I64))
        out = _Out(self.out.data_ptr(), self.out_off.ctypes.data_as(I64),
                   self.bond.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        self.stats.profile = 0
        _check(lib().cbc_apply_noalloc(self.ctx.h, ctypes.byref(ttno), ctypes.byref(ttns),
                                       ctypes.byref(self.tree.c), self.max_bond, float(tol),
                                       self.prec, ctypes.byref(out), ctypes.c_void_p(stream),
                                       ctypes.byref(self.stats)), "cbc_apply_noalloc")
        return self.out, self.bond

    def report(self, instance=0, stream=None, capacity=4096):
        """What the last call recorded on the device (waits for `stream`, default: the current
        one): {"status", "dropped_pivots", "trunc": [record dicts]}."""
        import torch
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        recs = (TruncRecord * capacity)()
        rep = Report(0, 0, 0, capacity, ctypes.cast(recs, ctypes.POINTER(TruncRecord)))
        rc = lib().cbc_read_report(self.workspace.data_ptr(), self.ws_bytes // self.batch,
                                   int(instance), ctypes.c_void_p(stream), ctypes.byref(rep))
        if rc not in (0, -5, -8):
            _check(rc, "cbc_read_report")
        trunc = [{f: getattr(recs[i], f) for f, _ in TruncRecord._fields_}
                 for i in range(min(rep.n_trunc, capacity))]
        return {"status": STATUS.get(rep.status, rep.status), "status_code": int(rep.status),
                "dropped_pivots": int(rep.dropped_pivots), "trunc": trunc}

    def check(self, instance=0, stream=None):
        """Raise if the device recorded a failure (non-finite factorisation, expired wait)."""
        r = self.report(instance, stream, capacity=0)
        if r["status_code"] != 0:
            _check(r["status_code"], "device")
        return r

    def unpack(self, instance=0):
        """Output node tensors as numpy complex128 arrays (sigma', parent bond, child bonds...).
        Synchronises the device (the library's calls are asynchronous)."""
        import torch
        torch.cuda.synchronize()
        total = int(self.out_off[-1])
        host = self.out[instance * total:(instance + 1) * total].cpu().numpy()
        res = []
        for i in range(self.tree.n):
            shape = (int(self.tree.phys[i]), int(self.bond[i])) + tuple(
                int(self.bond[c]) for c in self.tree.children[i])
            a, b = int(self.out_off[i]), int(self.out_off[i]) + int(np.prod(shape))
            res.append(host[a:b].reshape(shape))
        return res


def graph_groups(launches, cap):
    """Consecutive groups of instances whose kernel launches add up to at most `cap` (an instance
    above `cap` forms a group of its own); returns lists of instance indices."""
    groups, cur, n = [], [], 0
    for k, m in enumerate(launches):
        if cur and n + m > cap:
            groups.append(cur)
            cur, n = [], 0
        cur.append(k)
        n += m
    if cur:
        groups.append(cur)
    return groups


class CProblem(ctypes.Structure):
    _fields_ = [("tree", ctypes.POINTER(_Tree)), ("ttno", ctypes.POINTER(_Tensors)),
                ("ttns", ctypes.POINTER(_Tensors)), ("max_bond", ctypes.c_int32),
                ("tol", ctypes.c_double), ("workspace", ctypes.c_void_p),
                ("workspace_bytes", ctypes.c_size_t), ("out", ctypes.POINTER(_Out)),
                ("stats", ctypes.POINTER(Stats))]


class UnevenBatch:
    """Many instances of different shapes launched by cbc_apply_many: one Compressor (plan,
    workspace, outputs) per instance; the library spreads them round-robin over `nstreams` streams
    of its context, forked from and joined into the caller's stream. Inputs are packed once and stay
    resident. With `share_scratch`, the instances of one stream share one scratch buffer (their
    calls are ordered by the stream), sized for the largest of them: device memory is then the sum
    of the small persistent parts plus `nstreams` scratch buffers, instead of the sum of every
    instance's whole workspace."""

    def __init__(self, problems, precision="mixed", nstreams=8, device="cuda", autotune=False,
                 share_scratch=False):
        import torch
        self.ctx = Context()
        if autotune:
            self.ctx.autotune()
        self.nstreams = int(nstreams)
        self.prec = PRECISIONS[precision]
        trees = [Tree.of(p) for p in problems]
        self.scratch = []
        if share_scratch:
            # every stream's buffer fits every instance, so that a call over any consecutive range
            # of the instances (graphs of part of the batch) may use them
            need = max([scratch_need(self.ctx, t, p.max_bond, precision)["scratch_bytes"]
                        for p, t in zip(problems, trees)] + [256])
            self.scratch = [torch.empty(need, dtype=torch.uint8, device=device)
                            for _ in range(self.nstreams)]
        self.items = []
        self._keep = []
        self._problems = (CProblem * len(problems))()
        I64 = ctypes.POINTER(ctypes.c_int64)
        for k, (p, tree) in enumerate(zip(problems, trees)):
            st, so = pack(p.state, device)
            op, oo = pack(p.op, device)
            comp = Compressor(self.ctx, tree, p.max_bond, precision, device=device,
                              scratch=self.scratch[0] if share_scratch else None)
            self.items.append((comp, (op, oo, st, so, p.tol)))
            oo = np.ascontiguousarray(oo, dtype=np.int64)
            so = np.ascontiguousarray(so, dtype=np.int64)
            ttno = _Tensors(op.data_ptr(), oo.ctypes.data_as(I64))
            ttns = _Tensors(st.data_ptr(), so.ctypes.data_as(I64))
            out = _Out(comp.out.data_ptr(), comp.out_off.ctypes.data_as(I64),
                       comp.bond.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
            self._keep += [oo, so, ttno, ttns, out]
            self._problems[k] = CProblem(ctypes.pointer(tree.c), ctypes.pointer(ttno),
                                         ctypes.pointer(ttns), comp.max_bond, float(p.tol),
                                         comp.workspace.data_ptr(), comp.ws_bytes,
                                         ctypes.pointer(out), ctypes.pointer(comp.stats))
        if share_scratch:
            self._scr = (ctypes.c_void_p * self.nstreams)(*[x.data_ptr() for x in self.scratch])
            self._scr_bytes = (ctypes.c_size_t * self.nstreams)(*[x.numel() for x in self.scratch])
        else:
            self._scr = self._scr_bytes = None

    def run_range(self, lo, hi, stream=None):
        """Launch instances lo..hi-1 with one cbc_apply_many call on `stream` (default: the current
        stream); asynchronous."""
        import torch
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        if hi <= lo:
            return
        first = ctypes.cast(ctypes.byref(self._problems, lo * ctypes.sizeof(CProblem)),
                            ctypes.POINTER(CProblem))
        _check(lib().cbc_apply_many(self.ctx.h, hi - lo, first, self.prec, self.nstreams,
                                    self._scr, self._scr_bytes, ctypes.c_void_p(stream)),
               "cbc_apply_many")

    def run(self):
        """Launch every instance (asynchronous); call torch.cuda.synchronize() to wait."""
        if getattr(self, "graphs", None):
            for g in self.graphs:
                g.replay()
            return
        self.run_range(0, len(self.items))

    # Kernel launches recorded into one graph at most. Graphs of up to about 10,500 launches (16
    # instances of the uneven draw) replay correctly on MI355X; one graph of the whole 256-instance
    # draw (about 159,000 launches) ended the process with a segmentation fault at its first
    # replay, so larger batches are recorded as several graphs of at most this many launches.
    MAX_GRAPH_LAUNCHES = 12000

    def capture(self, graph=None, max_launches=None):
        """Record the batch into graphs of at most `max_launches` kernel launches each (default
        MAX_GRAPH_LAUNCHES; consecutive instances, at least one per graph), each holding one
        cbc_apply_many call (fork over the library's streams, the instances, join); run() then
        replays them in order, one launch each. Runs the batch once first, eagerly. `graph`: a
        torch.cuda.CUDAGraph to capture into when the batch fits one graph (default: a new one)."""
        import torch
        cap = self.MAX_GRAPH_LAUNCHES if max_launches is None else int(max_launches)
        self.graphs = []
        self.run()
        torch.cuda.synchronize()
        groups = graph_groups([int(comp.stats.n_kernels) for comp, _ in self.items], cap)
        if graph is not None and len(groups) > 1:
            raise ValueError("the batch needs several graphs; capture without `graph`")
        root = torch.cuda.Stream()
        graphs = []
        for grp in groups:
            g = graph if graph is not None else torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, stream=root):
                self.run_range(grp[0], grp[-1] + 1, root.cuda_stream)
            graphs.append(g)
        self.graphs = graphs

    def flops(self):
        return sum(c.stats.flops[0] for c, _ in self.items)


def plan_bonds(tree, max_bond, tol_on=False, ctx=None):
    """Output bond to the parent of every node as planned for `max_bond` (host only, no device)."""
    ctx = ctx or Context()
    bond = np.zeros(tree.n, dtype=np.int32)
    _check(lib().cbc_plan_bonds(ctx.h, ctypes.byref(tree.c), int(max_bond), int(bool(tol_on)),
                                bond.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))),
           "cbc_plan_bonds")
    return [int(b) for b in bond]


def scratch_need(ctx, tree, max_bond, precision):
    """Persistent and scratch bytes a cbc_apply_split call needs with or without a tolerance."""
    a = plan_info(tree, max_bond, precision, tol_on=False, ctx=ctx)
    b = plan_info(tree, max_bond, precision, tol_on=True, ctx=ctx)
    return {k: max(a[k], b[k]) for k in ("persistent_bytes", "scratch_bytes")}


def plan_info(tree, max_bond, precision="fp64", method="cbc", tol_on=False, ctx=None):
    """Planned workspace split and per-class launches and flops of one call (host only)."""
    ctx = ctx or Context()
    info = PlanSummary()
    _check(lib().cbc_plan_info(ctx.h, ctypes.byref(tree.c), int(max_bond), PRECISIONS[precision],
                               METHODS[method], int(bool(tol_on)), ctypes.byref(info)),
           "cbc_plan_info")
    return {"persistent_bytes": int(info.persistent_bytes), "scratch_bytes": int(info.scratch_bytes),
            "table_bytes": int(info.table_bytes),
            "launches": {c: int(info.launches[k]) for k, c in enumerate(CLASSES)},
            "flops": {c: float(info.flops[k]) for k, c in enumerate(CLASSES)}}


def compress(problem, precision="fp64", method="cbc", tol=None, ctx=None, device="cuda",
             sketch=None):
    """Convenience wrapper: one compression of a Problem from paper_2601_19650_amd.inputs.
    `sketch`: the randomised method's matrices (one d_i x max_bond numpy array per node)."""
    ctx = ctx or Context()
    tree = Tree.of(problem)
    st, so = pack(problem.state, device)
    op, oo = pack(problem.op, device)
    c = Compressor(ctx, tree, problem.max_bond, precision, method, device)
    sk = pack(sketch, device) if sketch is not None else None
    c.run(op, oo, st, so, problem.tol if tol is None else tol, sketch=sk)
    out = c.unpack()
    c.check()
    return out, c


# ------------------------------------------------------------------------------------------------
# kernel-level test entry points (include/cbc_testing.h)

def _testing_lib():
    L = lib()
    if not getattr(L, "_testing_ready", False):
        vp, ci, cd = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
        L.cbc_test_gemm.argtypes = [ci, ci, ci, vp, ci, ci, ci, vp, ci, ci, ci, vp, ci, ci, ci, vp]
        L.cbc_test_gemm.restype = ci
        L.cbc_test_eig.argtypes = [vp, ci, ci, cd, vp, vp, vp, vp, vp, vp]
        L.cbc_test_eig.restype = ci
        L.cbc_test_chol_inv.argtypes = [vp, ci, cd, cd, vp, vp, vp, vp]
        L.cbc_test_chol_inv.restype = ci
        L.cbc_test_gemm_time.argtypes = [ci, ci, ci, ci, ci, ci, ci, ci, ci,
                                         ctypes.POINTER(ctypes.c_float)]
        L.cbc_test_gemm_time.restype = ci
        L.cbc_test_eig_report.argtypes = [vp, ci, ci, cd, ci, vp, vp, vp, vp, vp, vp, vp]
        L.cbc_test_eig_reduction.argtypes = [vp, ci, ci, cd, ci, vp, vp, vp, vp, vp, vp]
        L.cbc_test_eig_reduction.restype = ci
        L.cbc_test_eig_report.restype = ci
        L._testing_ready = True
    return L


TESTING_EXPORTED = ("cbc_test_gemm", "cbc_test_gemm_time", "cbc_test_eig", "cbc_test_chol_inv",
                    "cbc_test_eig_report", "cbc_test_eig_reduction")


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def test_gemm(A, B, transA=False, conjA=False, transB=False, conjB=False, out_dtype=None,
              acc_fp64=True, tile=0):
    """C = op(A) op(B) on the GPU contraction kernel; A, B are torch complex device matrices."""
    import torch
    M = A.shape[1] if transA else A.shape[0]
    K = A.shape[0] if transA else A.shape[1]
    N = B.shape[0] if transB else B.shape[1]
    out_dtype = out_dtype or (torch.complex128 if acc_fp64 else torch.complex64)
    C = torch.empty((M, N), dtype=out_dtype, device=A.device)
    A = A.contiguous()
    B = B.contiguous()
    _check(_testing_lib().cbc_test_gemm(M, N, K, A.data_ptr(), int(A.dtype == torch.complex128),
                                        int(transA), int(conjA), B.data_ptr(),
                                        int(B.dtype == torch.complex128), int(transB), int(conjB),
                                        C.data_ptr(), int(out_dtype == torch.complex128),
                                        int(acc_fp64), int(tile), _stream()), "cbc_test_gemm")
    return C


def test_gemm_time(M, N, K, a_c128=False, b_c128=False, c_c128=False, acc_fp64=False, tile=-1,
                   reps=10):
    """Average milliseconds per launch of the contraction kernel on a plain M x N x K product."""
    ms = ctypes.c_float()
    _check(_testing_lib().cbc_test_gemm_time(M, N, K, int(a_c128), int(b_c128), int(c_c128),
                                             int(acc_fp64), int(tile), int(reps), ctypes.byref(ms)),
           "cbc_test_gemm_time")
    return float(ms.value)


def test_eig(G, kmax, tol=0.0, stamps=None, reduction=0):
    """Top-kmax eigenpairs of a Hermitian complex128 device matrix (G is consumed). If `stamps` is a
    list, the phase durations in microseconds are appended to it. `reduction` selects the reduction
    to tridiagonal form for s > 128 (0: two-stage, 1: one-stage multi-workgroup)."""
    import torch
    s = G.shape[0]
    G = G.contiguous().clone()
    U = torch.empty((s, kmax), dtype=torch.complex128, device=G.device)
    lam = torch.empty(kmax, dtype=torch.float64, device=G.device)
    kk = torch.empty(1, dtype=torch.int32, device=G.device)
    inv = torch.empty(1, dtype=torch.float64, device=G.device)
    ts = torch.zeros(16, dtype=torch.int64, device=G.device)
    _check(_testing_lib().cbc_test_eig_reduction(G.data_ptr(), s, kmax, float(tol), int(reduction),
                                                 U.data_ptr(), lam.data_ptr(), kk.data_ptr(),
                                                 inv.data_ptr(),
                                                 ts.data_ptr() if stamps is not None else None,
                                                 _stream()),
           "cbc_test_eig_reduction")
    if stamps is not None:
        t = ts.cpu().numpy()
        # tridiagonal, eigenvalues (incl. launch), eigenvectors (incl. launch), then the
        # tridiagonal step phases A/B/D and the number of clusters
        stamps.append([(t[1] - t[0]) / 100.0, (t[2] - t[1]) / 100.0, (t[3] - t[2]) / 100.0,
                       t[4] / 100.0, t[5] / 100.0, t[6] / 100.0, float(t[7])] +
                      [x / 100.0 for x in t[8:16]])
    return U, lam, int(kk.item()), float(inv.item())


def test_eig_report(G, kmax, tol=0.0, force_timeout=False):
    """Eigensolve with a status word and a truncation record (see cbc_test_eig_report); returns
    (status code, record dict, U, lam, kept)."""
    import torch
    s = G.shape[0]
    G = G.contiguous().clone()
    U = torch.empty((s, kmax), dtype=torch.complex128, device=G.device)
    lam = torch.empty(kmax, dtype=torch.float64, device=G.device)
    kk = torch.empty(1, dtype=torch.int32, device=G.device)
    inv = torch.empty(1, dtype=torch.float64, device=G.device)
    status = torch.zeros(1, dtype=torch.int32, device=G.device)
    rec = torch.zeros(ctypes.sizeof(TruncRecord), dtype=torch.uint8, device=G.device)
    _check(_testing_lib().cbc_test_eig_report(G.data_ptr(), s, kmax, float(tol), int(force_timeout),
                                              U.data_ptr(), lam.data_ptr(), kk.data_ptr(),
                                              inv.data_ptr(), status.data_ptr(), rec.data_ptr(),
                                              _stream()), "cbc_test_eig_report")
    r = TruncRecord.from_buffer_copy(bytes(rec.cpu().numpy()))
    return (int(status.item()), {f: getattr(r, f) for f, _ in TruncRecord._fields_}, U, lam,
            int(kk.item()))


def test_chol_inv(G, shift_rel=0.0, drop_rel=0.0, stamps=None):
    import torch
    k = G.shape[0]
    G = G.contiguous().clone()
    Ci = torch.empty((k, k), dtype=torch.complex128, device=G.device)
    nd = torch.zeros(1, dtype=torch.int32, device=G.device)
    ts = torch.zeros(4, dtype=torch.int64, device=G.device)
    _check(_testing_lib().cbc_test_chol_inv(G.data_ptr(), k, float(shift_rel), float(drop_rel),
                                            Ci.data_ptr(), nd.data_ptr(),
                                            ts.data_ptr() if stamps is not None else None, _stream()),
           "cbc_test_chol_inv")
    if stamps is not None:
        t = ts.cpu().numpy()
        stamps.append([(t[i + 1] - t[i]) / 100.0 for i in range(3)])
    return Ci, int(nd.item())
