"""ctypes wrapper of liboracle.so (plain C FP64 oracle).  Test infrastructure only."""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

KINDS = {"coulomb": 0, "yukawa": 1, "oscillatory": 2, "regcoulomb": 3, "poly": 100}
DEFAULT_PARAM = {"coulomb": 0.0, "yukawa": 0.5, "oscillatory": 0.0, "regcoulomb": 0.005, "poly": 0.0}
TYPES = ("PP", "PC", "CP", "CC")
# list-building methods: Algorithm 2, its PP+CC-only ablation (Sec. 4.3), and
# the two treecodes the paper compares with (BLTC, Sec. 2.8; CP-BLTC, Sec. 4.5)
SCHEMES = {"bldtt": 0, "pp_cc_only": 1, "bltc": 2, "cp_bltc": 3}

_lib = None
_D = C.POINTER(C.c_double)
_I64 = C.POINTER(C.c_int64)
_I32 = C.POINTER(C.c_int32)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = C.CDLL(_build.LIB)
        v = C.c_void_p
        L.or_direct_sum.argtypes = [C.c_int, C.c_double, C.c_int64, _D, _D, _D, C.c_int64, _D, _D, _D, _D,
                                    C.c_int64, _I64, _D]
        L.or_cheb.argtypes = [C.c_int, _D, _D]
        L.or_basis1d.argtypes = [C.c_int, C.c_double, C.c_double, C.c_double, _D]
        L.or_tree_build.restype = v
        L.or_tree_build.argtypes = [C.c_int64, _D, _D, _D, C.c_int64]
        L.or_tree_free.argtypes = [v]
        L.or_tree_size.restype = C.c_int64
        L.or_tree_size.argtypes = [v]
        L.or_tree_depth.restype = C.c_int32
        L.or_tree_depth.argtypes = [v]
        L.or_tree_export.argtypes = [v, _D, _D, _D, _D, _I64, _I64, _I64, _I32, _I32, _I64, _I64]
        L.or_lists_count.restype = C.c_int64
        L.or_lists_count.argtypes = [v, C.c_int]
        L.or_lists_export.argtypes = [v, C.c_int, _I64, _I64]
        L.or_run_create.restype = v
        L.or_run_create.argtypes = [C.c_int, C.c_double, C.c_int64, _D, _D, _D, C.c_int64, _D, _D, _D, _D,
                                    C.c_double, C.c_int, C.c_int64, C.c_int]
        L.or_run_free.argtypes = [v]
        L.or_run_tree.restype = v
        L.or_run_tree.argtypes = [v, C.c_int]
        L.or_run_lists.restype = v
        L.or_run_lists.argtypes = [v]
        for f in ("or_run_traverse", "or_run_upward", "or_run_interact", "or_run_downward", "or_run_all"):
            getattr(L, f).argtypes = [v]
        for f in ("or_run_upward_direct", "or_run_downward_direct", "or_run_potentials", "or_run_phi_tree",
                  "or_run_qhat", "or_run_phihat", "or_run_phihat_own", "or_run_times"):
            getattr(L, f).argtypes = [v, _D]
        L.or_run_eval_targets.argtypes = [v, C.c_int64, _I64, _D]
        L.or_run_interact_sample.restype = C.c_double
        L.or_run_interact_sample.argtypes = [v, C.c_int64, C.c_int64]
        L.or_run_eval_degrees.argtypes = [v, _I64, C.POINTER(_I64), C.POINTER(_I64), C.POINTER(_I32), _D]
        L.or_num_threads.restype = C.c_int
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(_D)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def num_threads() -> int:
    return int(lib().or_num_threads())


def direct_sum(tgt, src, kernel="coulomb", param=None, sel=None) -> np.ndarray:
    """Compensated FP64 direct sum at all targets, or at caller indices `sel`."""
    param = DEFAULT_PARAM[kernel] if param is None else param
    tx, ty, tz = (_f64(a) for a in (tgt.x, tgt.y, tgt.z))
    sx, sy, sz, q = (_f64(a) for a in (src.x, src.y, src.z, src.q))
    if sel is None:
        out = np.empty(tx.shape[0])
        lib().or_direct_sum(KINDS[kernel], param, tx.shape[0], _d(tx), _d(ty), _d(tz), sx.shape[0],
                            _d(sx), _d(sy), _d(sz), _d(q), 0, None, _d(out))
    else:
        sel = np.ascontiguousarray(sel, dtype=np.int64)
        out = np.empty(sel.shape[0])
        lib().or_direct_sum(KINDS[kernel], param, tx.shape[0], _d(tx), _d(ty), _d(tz), sx.shape[0],
                            _d(sx), _d(sy), _d(sz), _d(q), sel.shape[0], sel.ctypes.data_as(_I64), _d(out))
    return out


def cheb(n: int):
    xi = np.empty(n + 1)
    w = np.empty(n + 1)
    lib().or_cheb(n, _d(xi), _d(w))
    return xi, w


def basis1d(n: int, lo: float, hi: float, y: float) -> np.ndarray:
    L = np.empty(n + 1)
    lib().or_basis1d(n, lo, hi, y, _d(L))
    return L


def _export_tree(ptr, npart: int) -> dict:
    L = lib()
    nc = int(L.or_tree_size(ptr))
    lo = np.empty((nc, 3)); hi = np.empty((nc, 3)); center = np.empty((nc, 3)); radius = np.empty(nc)
    begin = np.empty(nc, np.int64); count = np.empty(nc, np.int64); parent = np.empty(nc, np.int64)
    level = np.empty(nc, np.int32); nchild = np.empty(nc, np.int32); child = np.empty((nc, 8), np.int64)
    perm = np.empty(npart, np.int64)
    L.or_tree_export(ptr, _d(lo), _d(hi), _d(center), _d(radius), begin.ctypes.data_as(_I64),
                     count.ctypes.data_as(_I64), parent.ctypes.data_as(_I64), level.ctypes.data_as(_I32),
                     nchild.ctypes.data_as(_I32), child.ctypes.data_as(_I64), perm.ctypes.data_as(_I64))
    return dict(lo=lo, hi=hi, center=center, radius=radius, begin=begin, count=count, parent=parent,
                level=level, nchild=nchild, child=child, perm=perm, depth=int(L.or_tree_depth(ptr)))


def build_tree(pset, leaf: int) -> dict:
    """Tree of one particle set (Sec. 2.3) as numpy arrays."""
    x, y, z = (_f64(a) for a in (pset.x, pset.y, pset.z))
    ptr = lib().or_tree_build(x.shape[0], _d(x), _d(y), _d(z), leaf)
    try:
        return _export_tree(ptr, x.shape[0])
    finally:
        lib().or_tree_free(ptr)


class Run:
    """One oracle BLDTT run; keeps the inputs alive for the C side."""

    def __init__(self, tgt, src, kernel="coulomb", theta=0.7, degree=6, leaf=500, param=None,
                 pp_cc_only=False, aliased=None, scheme="bldtt"):
        if pp_cc_only:
            scheme = "pp_cc_only"
        self.scheme = scheme
        self.kernel = kernel
        self.param = DEFAULT_PARAM[kernel] if param is None else param
        self.n = degree
        self.P = (degree + 1) ** 3
        if aliased is None:
            aliased = tgt is src
        self._s = [_f64(a) for a in (src.x, src.y, src.z, src.q)]
        self._t = self._s[:3] if aliased else [_f64(a) for a in (tgt.x, tgt.y, tgt.z)]
        self.M = self._t[0].shape[0]
        self.N = self._s[0].shape[0]
        tx, ty, tz = self._t
        sx, sy, sz, q = self._s
        self.ptr = lib().or_run_create(KINDS[kernel], self.param, self.M, _d(tx), _d(ty), _d(tz), self.N,
                                       _d(sx), _d(sy), _d(sz), _d(q), theta, degree, leaf, SCHEMES[scheme])
        self._lists = None

    def __del__(self):
        try:
            if getattr(self, "ptr", None):
                lib().or_run_free(self.ptr)
                self.ptr = None
        except Exception:
            pass

    def tree(self, which: int) -> dict:
        return _export_tree(lib().or_run_tree(self.ptr, which), self.N if which else self.M)

    def traverse(self):
        lib().or_run_traverse(self.ptr)
        self._lists = None

    def upward(self):
        lib().or_run_upward(self.ptr)

    def interact(self):
        lib().or_run_interact(self.ptr)

    def downward(self):
        lib().or_run_downward(self.ptr)

    def interact_sample(self, stride: int, offset: int = 0) -> float:
        """Time (s) of the interaction step on the leaves and clusters whose index
        is `offset` modulo `stride` (needs traverse + upward; potentials partial)."""
        return float(lib().or_run_interact_sample(self.ptr, int(stride), int(offset)))

    def run_all(self):
        lib().or_run_all(self.ptr)
        self._lists = None
        return self.potentials()

    def lists(self) -> dict:
        if self._lists is None:
            L = lib()
            lp = L.or_run_lists(self.ptr)
            out = {}
            for k, name in enumerate(TYPES):
                n = int(L.or_lists_count(lp, k))
                tc = np.empty(n, np.int64)
                sc = np.empty(n, np.int64)
                if n:
                    L.or_lists_export(lp, k, tc.ctypes.data_as(_I64), sc.ctypes.data_as(_I64))
                out[name] = (tc, sc)
            self._lists = out
        return self._lists

    def _get(self, fn, size):
        out = np.empty(size)
        getattr(lib(), fn)(self.ptr, _d(out))
        return out

    def potentials(self):
        return self._get("or_run_potentials", self.M)

    def phi_tree(self):
        return self._get("or_run_phi_tree", self.M)

    def n_clusters(self, which):
        return int(lib().or_tree_size(lib().or_run_tree(self.ptr, which)))

    def qhat(self):
        return self._get("or_run_qhat", self.n_clusters(1) * self.P).reshape(-1, self.P)

    def qhat_direct(self):
        return self._get("or_run_upward_direct", self.n_clusters(1) * self.P).reshape(-1, self.P)

    def phihat(self):
        return self._get("or_run_phihat", self.n_clusters(0) * self.P).reshape(-1, self.P)

    def phihat_own(self):
        return self._get("or_run_phihat_own", self.n_clusters(0) * self.P).reshape(-1, self.P)

    def downward_direct(self):
        return self._get("or_run_downward_direct", self.M)

    def times(self):
        return dict(zip(("traverse", "upward", "interact", "downward"), self._get("or_run_times", 4)))

    def eval_degrees(self, lists: dict) -> np.ndarray:
        """Potentials (caller order) for lists whose PC/CP/CC entries carry their own degree:
        lists[name] = (tc, sc, deg) for name in PP, PC, CP, CC (deg ignored for PP)."""
        keep = []
        n = np.zeros(4, np.int64)
        tcs, scs, degs = (_I64 * 4)(), (_I64 * 4)(), (_I32 * 4)()
        for k, name in enumerate(TYPES):
            tc, sc, dg = lists[name]
            tc = np.ascontiguousarray(tc, np.int64)
            sc = np.ascontiguousarray(sc, np.int64)
            dg = np.ascontiguousarray(dg, np.int32)
            keep += [tc, sc, dg]
            n[k] = tc.shape[0]
            tcs[k] = tc.ctypes.data_as(_I64)
            scs[k] = sc.ctypes.data_as(_I64)
            degs[k] = dg.ctypes.data_as(_I32)
        out = np.empty(self.M)
        lib().or_run_eval_degrees(self.ptr, n.ctypes.data_as(_I64), tcs, scs, degs, _d(out))
        return out

    def eval_targets(self, sel) -> np.ndarray:
        """Potentials at caller-order targets `sel` (needs traverse + upward only)."""
        sel = np.ascontiguousarray(sel, dtype=np.int64)
        out = np.empty(sel.shape[0])
        lib().or_run_eval_targets(self.ptr, sel.shape[0], sel.ctypes.data_as(_I64), _d(out))
        return out


def bldtt(tgt, src, kernel="coulomb", theta=0.7, degree=6, leaf=500, param=None, pp_cc_only=False,
          aliased=None, scheme="bldtt") -> np.ndarray:
    """Potentials in caller order from a full oracle run (BLDTT unless `scheme` names a treecode)."""
    r = Run(tgt, src, kernel, theta, degree, leaf, param, pp_cc_only, aliased, scheme)
    return r.run_all()


def rel_l2(a, b) -> float:
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.sqrt(np.sum((a - b) ** 2) / np.sum(b ** 2)))


def max_rel(a, b) -> float:
    """max_i |a_i - b_i| / max_i |b_i|: an element-wise bound that a single
    wrong value cannot hide behind the norm (0 when both are all zero)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    d = float(np.max(np.abs(a - b))) if a.size else 0.0
    s = float(np.max(np.abs(b))) if b.size else 0.0
    return d / s if s > 0 else d
