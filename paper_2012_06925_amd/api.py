"""Thin Python binding of the BLDTT C ABI: argument marshalling only.

Every step of the compute phase runs in libbldtt.so (HIP kernels and the C++
host engine).  torch supplies device memory and the stream; nothing here
computes potentials.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib
from ._lib import KERNELS, DEFAULT_PARAM, TYPES, check, lib


def _f64_cuda(t: torch.Tensor, name: str) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda" or t.dtype != torch.float64:
        raise TypeError(f"{name} must be a float64 torch.cuda tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def _stream_ptr(stream) -> int:
    s = torch.cuda.current_stream() if stream is None else stream
    return int(s.cuda_stream)


def _kernel(kernel: str, param):
    if kernel not in KERNELS:
        raise ValueError(f"unknown kernel {kernel!r}")
    return KERNELS[kernel], DEFAULT_PARAM[kernel] if param is None else float(param)


def _tree_dict(view: _lib.TreeView) -> dict:
    nc, npart = view.n_clusters, view.n_particles

    def arr(p, n, dt):
        return np.ctypeslib.as_array(p, shape=(n,)).astype(dt, copy=True)

    return dict(lo=arr(view.lo, 3 * nc, np.float64).reshape(nc, 3), hi=arr(view.hi, 3 * nc, np.float64).reshape(nc, 3),
                center=arr(view.center, 3 * nc, np.float64).reshape(nc, 3), radius=arr(view.radius, nc, np.float64),
                begin=arr(view.begin, nc, np.int64), count=arr(view.count, nc, np.int64),
                parent=arr(view.parent, nc, np.int64), child=arr(view.child, 8 * nc, np.int64).reshape(nc, 8),
                perm=arr(view.perm, npart, np.int64), level=arr(view.level, nc, np.int32),
                nchild=arr(view.nchild, nc, np.int32), depth=int(view.depth))


class _PlanBase:
    _handle = None

    def close(self):
        if self._handle:
            check(lib().bldtt_destroy(self._handle))
            self._handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def tree(self, which: int = 0) -> dict:
        v = _lib.TreeView()
        check(lib().bldtt_get_tree(self._handle, which, C.byref(v)))
        return _tree_dict(v)

    def lists(self) -> dict:
        out = {}
        for k, name in enumerate(TYPES):
            tc, sc, n = _lib._I64(), _lib._I64(), C.c_int64()
            check(lib().bldtt_get_lists(self._handle, k, C.byref(tc), C.byref(sc), C.byref(n)))
            if n.value:
                out[name] = (np.ctypeslib.as_array(tc, shape=(n.value,)).copy(),
                             np.ctypeslib.as_array(sc, shape=(n.value,)).copy())
            else:
                out[name] = (np.empty(0, np.int64), np.empty(0, np.int64))
        return out

    def list_degrees(self) -> dict:
        out = {}
        for k, name in enumerate(TYPES):
            d, n = C.POINTER(C.c_int8)(), C.c_int64()
            check(lib().bldtt_get_list_degrees(self._handle, k, C.byref(d), C.byref(n)))
            out[name] = np.ctypeslib.as_array(d, shape=(n.value,)).astype(np.int32) if n.value else np.empty(0, np.int32)
        return out

    def stats(self) -> dict:
        s = _lib.Stats()
        check(lib().bldtt_get_stats(self._handle, C.byref(s)))
        return dict(n_entries=dict(zip(TYPES, list(s.n_entries))),
                    interactions=dict(zip(TYPES, list(s.interactions))),
                    n_target_clusters=s.n_target_clusters, n_source_clusters=s.n_source_clusters,
                    target_depth=s.target_depth, source_depth=s.source_depth, setup_ms=s.setup_ms,
                    traverse_ms=s.traverse_ms, compute_host_ms=s.compute_host_ms,
                    phase_ms=dict(zip(_lib.PHASES, list(s.phase_ms))), profiled_computes=s.profiled_computes,
                    down_degree=s.down_degree, degree_mask=s.degree_mask, sep_pairs=s.sep_pairs,
                    sep_fallback=s.sep_fallback, sep_direct=s.sep_direct,
                    pairs_per_degree={d: int(s.pairs_per_degree[d]) for d in range(13) if s.pairs_per_degree[d]},
                    pass_interactions=list(s.pass_interactions), host_marks_ms=list(s.host_marks_ms),
                    fp64_close_pairs=int(s.fp64_close_pairs))

    def traverse_host(self):
        check(lib().bldtt_traverse_host(self._handle))


class Plan(_PlanBase):
    """bldtt_setup on device tensors; compute() returns potentials in caller order.

    targets: (x, y, z) float64 cuda tensors, or None when targets = sources.
    sources: (x, y, z, q) float64 cuda tensors.
    """

    def __init__(self, targets, sources, kernel="coulomb", theta=0.7, degree=6, leaf=500, param=None, flags=0,
                 stream=None):
        sx, sy, sz, q = (_f64_cuda(t, n) for t, n in zip(sources, ("sx", "sy", "sz", "q")))
        if targets is None:
            tx, ty, tz = sx, sy, sz
        else:
            tx, ty, tz = (_f64_cuda(t, n) for t, n in zip(targets, ("tx", "ty", "tz")))
        kind, kparam = _kernel(kernel, param)
        self.M, self.N, self.degree = tx.numel(), sx.numel(), degree
        self.P = (degree + 1) ** 3
        self.device = sx.device
        p = _lib.Particles(self.M, tx.data_ptr(), ty.data_ptr(), tz.data_ptr(), self.N, sx.data_ptr(),
                           sy.data_ptr(), sz.data_ptr(), q.data_ptr())
        h = C.c_void_p()
        with torch.cuda.device(self.device):
            check(lib().bldtt_setup(C.byref(h), C.byref(p), kind, kparam, float(theta), int(degree), int(leaf),
                                    int(flags), _stream_ptr(stream)))
        self._handle = h

    def compute(self, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        if out is None:
            out = torch.empty(self.M, dtype=torch.float64, device=self.device)
        _f64_cuda(out, "out")
        if out.numel() != self.M:
            raise ValueError("out must hold M values")
        with torch.cuda.device(self.device):
            check(lib().bldtt_compute(self._handle, out.data_ptr(), _stream_ptr(stream)))
        return out

    def qhat(self) -> np.ndarray:
        n = self.stats()["n_source_clusters"]
        out = np.empty(n * self.P)
        check(lib().bldtt_get_qhat(self._handle, out.ctypes.data_as(_lib._D)))
        return out.reshape(n, self.P)

    def set_degree_model(self, model: np.ndarray | None, fallback: int = 8, tau: float = 1e-7):
        """Per-pair degree policy of a plan set up with LEARNED_DEGREE (model None: fallback degree everywhere)."""
        if model is None:
            check(lib().bldtt_set_degree_model(self._handle, None, 0, int(fallback), float(tau)))
            return
        m = np.ascontiguousarray(model, dtype=np.float32)
        check(lib().bldtt_set_degree_model(self._handle, m.ctypes.data, m.size, int(fallback), float(tau)))

    def set_degree_test_rule(self):
        check(lib().bldtt_set_degree_test_rule(self._handle))

    def pair_errors(self, stream=None, with_pairs=False):
        """(features[n, 4], log10 errors[n, 11][, pairs[n, 2]]) of every separated pair, measured on the GPU."""
        n = C.c_int64()
        f, e, pr = C.POINTER(C.c_float)(), C.POINTER(C.c_float)(), _lib._I64()
        with torch.cuda.device(self.device):
            check(lib().bldtt_pair_errors(self._handle, _stream_ptr(stream), C.byref(n), C.byref(f), C.byref(e),
                                          C.byref(pr)))
        if n.value == 0:
            out = (np.empty((0, 4), np.float32), np.empty((0, 11), np.float32), np.empty((0, 2), np.int64))
        else:
            out = (np.ctypeslib.as_array(f, shape=(n.value, 4)).copy(),
                   np.ctypeslib.as_array(e, shape=(n.value, 11)).copy(),
                   np.ctypeslib.as_array(pr, shape=(n.value, 2)).copy())
        return out if with_pairs else out[:2]

    def phihat(self) -> np.ndarray:
        n = self.stats()["n_target_clusters"]
        out = np.empty(n * self.P)
        check(lib().bldtt_get_phihat(self._handle, out.ctypes.data_as(_lib._D)))
        return out.reshape(n, self.P)


class HostPlan(_PlanBase):
    """bldtt_setup_host on numpy arrays: trees and traversal only, no device."""

    def __init__(self, targets, sources, kernel="coulomb", theta=0.7, degree=6, leaf=500, param=None, flags=0):
        def f64(a):
            return np.ascontiguousarray(a, dtype=np.float64)

        self._keep = [f64(a) for a in sources]
        sx, sy, sz, q = self._keep
        if targets is None:
            tx, ty, tz = sx, sy, sz
        else:
            self._keep += [f64(a) for a in targets]
            tx, ty, tz = self._keep[4:7]
        kind, kparam = _kernel(kernel, param)
        p = _lib.Particles(tx.shape[0], tx.ctypes.data, ty.ctypes.data, tz.ctypes.data, sx.shape[0], sx.ctypes.data,
                           sy.ctypes.data, sz.ctypes.data, q.ctypes.data)
        h = C.c_void_p()
        check(lib().bldtt_setup_host(C.byref(h), C.byref(p), kind, kparam, float(theta), int(degree), int(leaf),
                                     int(flags)))
        self._handle = h


def direct_sum(targets, sources, kernel="coulomb", param=None, sel: torch.Tensor | None = None, stream=None):
    """Compensated FP64 direct sum (Eq. 1) at all targets or at caller indices `sel` (int64 cuda tensor)."""
    tx, ty, tz = (_f64_cuda(t, n) for t, n in zip(targets, ("tx", "ty", "tz")))
    sx, sy, sz, q = (_f64_cuda(t, n) for t, n in zip(sources, ("sx", "sy", "sz", "q")))
    kind, kparam = _kernel(kernel, param)
    if sel is not None:
        if sel.dtype != torch.int64 or sel.device.type != "cuda":
            raise TypeError("sel must be an int64 cuda tensor")
        n = sel.numel()
        selp = sel.data_ptr()
    else:
        n = tx.numel()
        selp = None
    out = torch.empty(n, dtype=torch.float64, device=sx.device)
    with torch.cuda.device(sx.device):
        check(lib().bldtt_direct_sum(kind, kparam, tx.numel(), tx.data_ptr(), ty.data_ptr(), tz.data_ptr(),
                                     sx.numel(), sx.data_ptr(), sy.data_ptr(), sz.data_ptr(), q.data_ptr(), n,
                                     selp, out.data_ptr(), _stream_ptr(stream)))
    return out


def set_tune_cache(path: str | None) -> None:
    """File that holds the autotuner's choices (None: memory only)."""
    check(lib().bldtt_set_tune_cache(None if path is None else str(path).encode()))


def autotune(plan: Plan, reps: int = 2, stream=None) -> None:
    """Time every tile pair on `plan`, keep the fastest, store it in the tune cache."""
    scratch = torch.empty(plan.M, dtype=torch.float64, device=plan.device)
    with torch.cuda.device(plan.device):
        check(lib().bldtt_autotune(plan._handle, scratch.data_ptr(), int(reps), _stream_ptr(stream)))


class Batch:
    """bldtt_batch_setup: many independent targets = sources (or separate)
    problems in one persistent, graph-captured launch.

    problems: list of (targets, sources) pairs as for Plan (targets None when
    targets = sources).  compute() returns one potentials tensor per problem.
    """

    _handle = None

    def __init__(self, problems, kernel="coulomb", theta=0.7, degree=6, leaf=500, param=None, flags=0, stream=None):
        kind, kparam = _kernel(kernel, param)
        arr = (_lib.Particles * len(problems))()
        self.M = []
        self._keep = []
        for i, (targets, sources) in enumerate(problems):
            sx, sy, sz, q = (_f64_cuda(t, n) for t, n in zip(sources, ("sx", "sy", "sz", "q")))
            if targets is None:
                tx, ty, tz = sx, sy, sz
            else:
                tx, ty, tz = (_f64_cuda(t, n) for t, n in zip(targets, ("tx", "ty", "tz")))
            arr[i] = _lib.Particles(tx.numel(), tx.data_ptr(), ty.data_ptr(), tz.data_ptr(), sx.numel(),
                                    sx.data_ptr(), sy.data_ptr(), sz.data_ptr(), q.data_ptr())
            self.M.append(tx.numel())
            self.device = sx.device
        h = C.c_void_p()
        with torch.cuda.device(self.device):
            check(lib().bldtt_batch_setup(C.byref(h), len(problems), arr, kind, kparam, float(theta), int(degree),
                                          int(leaf), int(flags), _stream_ptr(stream)))
        self._handle = h

    def compute(self, outs=None, stream=None):
        if outs is None:
            outs = [torch.empty(m, dtype=torch.float64, device=self.device) for m in self.M]
        if len(outs) != len(self.M):
            raise ValueError("one output tensor per problem")
        ptrs = (C.c_void_p * len(outs))()
        for i, (o, m) in enumerate(zip(outs, self.M)):
            _f64_cuda(o, "out")
            if o.numel() != m:
                raise ValueError(f"output {i} must hold {m} values")
            ptrs[i] = o.data_ptr()
        with torch.cuda.device(self.device):
            check(lib().bldtt_batch_compute(self._handle, ptrs, _stream_ptr(stream)))
        return outs

    def check(self, stream=None):
        with torch.cuda.device(self.device):
            check(lib().bldtt_batch_check(self._handle, _stream_ptr(stream)))

    def tune(self, reps: int = 3, stream=None):
        with torch.cuda.device(self.device):
            check(lib().bldtt_batch_tune(self._handle, int(reps), _stream_ptr(stream)))

    def set_tile(self, tpt: int, groups_per_cu: int = 0):
        with torch.cuda.device(self.device):
            check(lib().bldtt_batch_set_tile(self._handle, int(tpt), int(groups_per_cu)))

    def set_spin_limit(self, limit: int):
        with torch.cuda.device(self.device):
            check(lib().bldtt_batch_set_spin_limit(self._handle, int(limit)))

    def stats(self) -> dict:
        s = _lib.BatchStats()
        check(lib().bldtt_batch_get_stats(self._handle, C.byref(s)))
        out = {name: getattr(s, name) for name, _ in s._fields_ if name not in ("n_entries", "interactions")}
        out["n_entries"] = dict(zip(TYPES, list(s.n_entries)))
        out["interactions"] = dict(zip(TYPES, list(s.interactions)))
        return out

    def close(self):
        if self._handle:
            check(lib().bldtt_batch_destroy(self._handle))
            self._handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class HostBatch:
    """bldtt_batch_setup_host on host (numpy) arrays: the forest, its traversal
    and work items, with no device use.  problems: list of (targets, sources)
    with targets (x, y, z) or None, sources (x, y, z, q) float64 arrays."""

    _handle = None

    def __init__(self, problems, kernel="coulomb", theta=0.7, degree=6, leaf=500, param=None, flags=0, tpt=2):
        kind, kparam = _kernel(kernel, param)
        arr = (_lib.Particles * len(problems))()
        self._keep = []
        for i, (targets, sources) in enumerate(problems):
            sx, sy, sz, q = (np.ascontiguousarray(a, dtype=np.float64) for a in sources)
            if targets is None:
                tx, ty, tz = sx, sy, sz
            else:
                tx, ty, tz = (np.ascontiguousarray(a, dtype=np.float64) for a in targets)
            self._keep += [sx, sy, sz, q, tx, ty, tz]
            ptr = lambda a: a.ctypes.data
            arr[i] = _lib.Particles(tx.size, ptr(tx), ptr(ty), ptr(tz), sx.size, ptr(sx), ptr(sy), ptr(sz), ptr(q))
        h = C.c_void_p()
        check(lib().bldtt_batch_setup_host(C.byref(h), len(problems), arr, kind, kparam, float(theta), int(degree),
                                           int(leaf), int(flags), int(tpt)))
        self._handle = h
        self._keep = []

    def tree(self, which: int = 0) -> dict:
        v = _lib.TreeView()
        check(lib().bldtt_batch_get_tree(self._handle, int(which), C.byref(v)))
        return _tree_dict(v)

    def lists(self) -> dict:
        out = {}
        for k, name in enumerate(TYPES):
            tc, sc, n = _lib._I64(), _lib._I64(), C.c_int64()
            check(lib().bldtt_batch_get_lists(self._handle, k, C.byref(tc), C.byref(sc), C.byref(n)))
            m = n.value
            a = np.ctypeslib.as_array(tc, shape=(m,)).copy() if m else np.zeros(0, np.int64)
            b = np.ctypeslib.as_array(sc, shape=(m,)).copy() if m else np.zeros(0, np.int64)
            out[name] = (a, b)
        return out

    def stats(self) -> dict:
        return Batch.stats(self)

    def compute_raw(self):
        """bldtt_batch_compute on this handle (returns the status; host-only batches refuse)."""
        ptrs = (C.c_void_p * 1)()
        return lib().bldtt_batch_compute(self._handle, ptrs, None)

    close = Batch.close
    __del__ = Batch.__del__
    __enter__ = Batch.__enter__
    __exit__ = Batch.__exit__


def mlp_model_size() -> int:
    return int(lib().bldtt_mlp_model_size())


def _f32_cuda(t, name):
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda" or t.dtype != torch.float32 or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous float32 cuda tensor")
    return t


def mlp_forward(model: torch.Tensor, features: torch.Tensor, stream=None) -> torch.Tensor:
    """Predicted log10 pair errors [n, 11] for features [n, 4] (device tensors)."""
    _f32_cuda(model, "model")
    _f32_cuda(features, "features")
    n = features.shape[0]
    out = torch.empty((n, 11), dtype=torch.float32, device=features.device)
    check(lib().bldtt_mlp_forward(model.data_ptr(), features.data_ptr(), n, out.data_ptr(), _stream_ptr(stream)))
    return out


def mlp_loss_grad(model: torch.Tensor, features: torch.Tensor, targets: torch.Tensor, stream=None):
    """(loss, gradient) of the mean squared error, computed by the GPU backward kernels."""
    for t, nm in ((model, "model"), (features, "features"), (targets, "targets")):
        _f32_cuda(t, nm)
    n = features.shape[0]
    grad = torch.empty(mlp_model_size() - 16, dtype=torch.float32, device=features.device)
    loss = torch.empty(1, dtype=torch.float32, device=features.device)
    check(lib().bldtt_mlp_loss_grad(model.data_ptr(), features.data_ptr(), targets.data_ptr(), n, grad.data_ptr(),
                                    loss.data_ptr(), _stream_ptr(stream)))
    return float(loss.item()), grad


def mlp_train(features: np.ndarray, targets: np.ndarray, epochs: int = 200, batch: int = 1024, lr: float = 2e-3,
              seed: int = 0, stream=None):
    """Train the degree model on the GPU; returns (model record, loss per epoch)."""
    f = np.ascontiguousarray(features, dtype=np.float32)
    t = np.ascontiguousarray(targets, dtype=np.float32)
    if f.ndim != 2 or f.shape[1] != 4 or t.shape != (f.shape[0], 11):
        raise ValueError("features must be [n, 4] and targets [n, 11]")
    model = np.empty(mlp_model_size(), dtype=np.float32)
    hist = np.empty(epochs, dtype=np.float32)
    check(lib().bldtt_mlp_train(f.ctypes.data, t.ctypes.data, f.shape[0], int(epochs), int(batch), float(lr),
                                int(seed), model.ctypes.data, hist.ctypes.data, _stream_ptr(stream)))
    return model, hist


_allocator_refs = None       # the registered ctypes callbacks, kept alive


def set_allocator(alloc, release) -> None:
    """Device memory of plans and batches from alloc(nbytes) -> int pointer (0 on
    failure) and release(pointer); both None restores hipMalloc / hipFree."""
    global _allocator_refs
    if alloc is None and release is None:
        check(lib().bldtt_set_allocator(None, None, None))
        _allocator_refs = None
        return

    def _alloc(n, _ctx):
        try:
            return int(alloc(int(n))) or None
        except Exception:            # a failed allocation is reported as NULL (BLDTT_ENOMEM)
            return None

    def _release(ptr, _ctx):
        release(int(ptr))

    refs = (_lib.ALLOC_FN(_alloc), _lib.RELEASE_FN(_release))
    check(lib().bldtt_set_allocator(C.cast(refs[0], C.c_void_p), C.cast(refs[1], C.c_void_p), None))
    _allocator_refs = refs


def use_torch_allocator() -> None:
    """Take the library's device memory from torch's caching allocator (the
    current device and stream of each call); the binding does this on import."""
    set_allocator(lambda n: torch.cuda.caching_allocator_alloc(n),
                  lambda ptr: torch.cuda.caching_allocator_delete(ptr))


def version() -> str:
    return lib().bldtt_version().decode()


use_torch_allocator()
