"""Host logic of the HIP library, on the CPU: the C ABI loads and exports every
declared symbol, argument errors are reported, and the library's own tree
build and traversal (C++ host engine) agree bit for bit with the oracle's."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from oracle import core
from paper_2012_06925_amd import inputs

api = pytest.importorskip("paper_2012_06925_amd.api")
from paper_2012_06925_amd import _lib  # noqa: E402

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    header = open(os.path.join(ROOT, "include", "bldtt.h")).read()
    declared = set(re.findall(r"^\s*(?:int|const char \*)\s*(bldtt_\w+)\s*\(", header, re.M))
    assert declared, "no declarations found"
    L = C.CDLL(_lib.LIB_PATH)
    for name in declared:
        assert hasattr(L, name), name
    # the binding knows every declared symbol and nothing else
    assert declared == set(_lib.SIGNATURES)
    assert "gfx950" in api.version()


def _same(tree_a, tree_b):
    for k in tree_a:
        if k == "depth":
            assert tree_a[k] == tree_b[k]
        else:
            assert np.array_equal(tree_a[k], tree_b[k]), k


def _same_lists(la, lb):
    for k in ("PP", "PC", "CP", "CC"):
        a = sorted(zip(*la[k]))
        b = sorted(zip(*lb[k]))
        assert a == b, k


@pytest.mark.parametrize("dist,n,theta,deg,leaf", [
    ("uniform", 10_000, 0.7, 6, 500),
    ("gaussian", 30_000, 0.8, 4, 100),
    ("sphere", 20_000, 0.5, 3, 64),
    ("rod", 15_000, 0.9, 2, 40),
    ("slab", 15_000, 0.7, 5, 80),
    ("plummer", 20_000, 0.7, 5, 100),
])
def test_trees_and_lists_bit_exact_same_set(dist, n, theta, deg, leaf):
    p = inputs.particles(n, dist, seed=31)
    hp = api.HostPlan(None, (p.x, p.y, p.z, p.q), theta=theta, degree=deg, leaf=leaf)
    hp.traverse_host()
    r = core.Run(p, p, theta=theta, degree=deg, leaf=leaf)
    r.traverse()
    _same(r.tree(0), hp.tree(0))
    _same_lists(r.lists(), hp.lists())
    st = hp.stats()
    assert st["n_entries"] == {k: len(v[0]) for k, v in r.lists().items()}


@pytest.mark.parametrize("ablation", [False, True])
def test_trees_and_lists_bit_exact_unequal(ablation):
    t, s = inputs.unequal_sets(25_000, "sphere", 40_000, "gaussian", seed=32)
    flags = _lib.PP_CC_ONLY if ablation else 0
    hp = api.HostPlan((t.x, t.y, t.z), (s.x, s.y, s.z, s.q), theta=0.7, degree=3, leaf=100, flags=flags)
    hp.traverse_host()
    r = core.Run(t, s, theta=0.7, degree=3, leaf=100, pp_cc_only=ablation)
    r.traverse()
    _same(r.tree(0), hp.tree(0))
    _same(r.tree(1), hp.tree(1))
    _same_lists(r.lists(), hp.lists())
    if ablation:
        L = hp.lists()
        assert len(L["PC"][0]) == 0 and len(L["CP"][0]) == 0


@pytest.mark.parametrize("scheme", ["bltc", "cp_bltc"])
@pytest.mark.parametrize("case", ["same", "unequal"])
def test_treecode_lists_bit_exact(scheme, case):
    # the library's BLTC / CP-BLTC walks (Sec. 2.8, Sec. 4.5) against the oracle's
    flags = _lib.BLTC if scheme == "bltc" else _lib.CP_BLTC
    if case == "same":
        t = s = inputs.particles(30_000, "gaussian", seed=35)
        hp = api.HostPlan(None, (s.x, s.y, s.z, s.q), theta=0.7, degree=3, leaf=100, flags=flags)
    else:
        t, s = inputs.unequal_sets(25_000, "sphere", 40_000, "gaussian", seed=36)
        hp = api.HostPlan((t.x, t.y, t.z), (s.x, s.y, s.z, s.q), theta=0.7, degree=3, leaf=100, flags=flags)
    hp.traverse_host()
    r = core.Run(t, s, theta=0.7, degree=3, leaf=100, scheme=scheme, aliased=case == "same")
    r.traverse()
    _same_lists(r.lists(), hp.lists())
    L = hp.lists()
    approx = "PC" if scheme == "bltc" else "CP"
    assert len(L[approx][0]) > 0
    assert all(len(L[k][0]) == 0 for k in ("PC", "CP", "CC") if k != approx)


def test_treecode_flag_errors():
    p = inputs.particles(2000, seed=37)
    src = (p.x, p.y, p.z, p.q)
    for bad in (_lib.BLTC | _lib.CP_BLTC, _lib.BLTC | _lib.PP_CC_ONLY, _lib.CP_BLTC | _lib.PP_CC_ONLY):
        with pytest.raises(_lib.BldttError) as e:
            api.HostPlan(None, src, theta=0.7, degree=3, leaf=100, flags=bad)
        assert e.value.code == _lib.EINVAL
    for scheme in (_lib.BLTC, _lib.CP_BLTC):
        with pytest.raises(_lib.BldttError) as e:
            api.HostPlan(None, src, theta=0.7, degree=3, leaf=100, flags=scheme | _lib.LEARNED_DEGREE)
        assert e.value.code == _lib.EUNSUPPORTED
        with pytest.raises(_lib.BldttError) as e:
            api.HostBatch([(None, src), (None, src)], theta=0.7, degree=3, leaf=100, flags=scheme)
        assert e.value.code == _lib.EUNSUPPORTED


def test_device_tree_flag_needs_a_device_plan():
    p = inputs.particles(2000, seed=38)
    with pytest.raises(_lib.BldttError) as e:
        api.HostPlan(None, (p.x, p.y, p.z, p.q), theta=0.7, degree=3, leaf=100, flags=_lib.DEVICE_TREE)
    assert e.value.code == _lib.EINVAL
    with pytest.raises(_lib.BldttError) as e:
        api.HostBatch([(None, (p.x, p.y, p.z, p.q))] * 2, theta=0.7, degree=3, leaf=100, flags=_lib.DEVICE_TREE)
    assert e.value.code == _lib.EUNSUPPORTED


def test_large_tree_parallel_build_bit_exact():
    # above the serial cutoff: the multi-threaded partition must give the same tree
    p = inputs.particles(400_000, "gaussian", seed=33)
    hp = api.HostPlan(None, (p.x, p.y, p.z, p.q), theta=0.7, degree=6, leaf=2000)
    hp.traverse_host()
    r = core.Run(p, p, theta=0.7, degree=6, leaf=2000)
    r.traverse()
    _same(r.tree(0), hp.tree(0))
    _same_lists(r.lists(), hp.lists())


def test_degenerate_geometries():
    n = 3000
    rng = np.random.default_rng(34)
    cases = {
        "identical": (np.full(n, 0.3), np.full(n, -0.2), np.full(n, 0.7)),
        "collinear": (rng.uniform(-1, 1, n), np.full(n, 0.1), np.full(n, 0.1)),
        "coplanar": (rng.uniform(-1, 1, n), rng.uniform(-1, 1, n), np.zeros(n)),
        "duplicates": tuple(np.repeat(rng.uniform(-1, 1, n // 3), 3) for _ in range(3)),
    }
    for name, (x, y, z) in cases.items():
        q = rng.uniform(-1, 1, x.shape[0])
        p = inputs.ParticleSet(x.copy(), y.copy(), z.copy(), q)
        hp = api.HostPlan(None, (p.x, p.y, p.z, p.q), theta=0.7, degree=3, leaf=50)
        hp.traverse_host()
        r = core.Run(p, p, theta=0.7, degree=3, leaf=50)
        r.traverse()
        _same(r.tree(0), hp.tree(0))
        _same_lists(r.lists(), hp.lists())


def test_single_particle_sets():
    one = inputs.ParticleSet(np.array([0.5]), np.array([0.5]), np.array([0.5]), np.array([1.0]))
    hp = api.HostPlan(None, (one.x, one.y, one.z, one.q), theta=0.7, degree=2, leaf=1)
    hp.traverse_host()
    L = hp.lists()
    assert list(zip(*L["PP"])) == [(0, 0)]


def _expect(code, fn):
    with pytest.raises(_lib.BldttError) as ei:
        fn()
    assert ei.value.code == code, str(ei.value)


def test_argument_errors():
    p = inputs.particles(100, seed=35)
    src = (p.x, p.y, p.z, p.q)
    _expect(_lib.EINVAL, lambda: api.HostPlan(None, src, theta=1.0))
    _expect(_lib.EINVAL, lambda: api.HostPlan(None, src, theta=0.0))
    _expect(_lib.EINVAL, lambda: api.HostPlan(None, src, degree=0))
    _expect(_lib.EINVAL, lambda: api.HostPlan(None, src, degree=13))
    _expect(_lib.EINVAL, lambda: api.HostPlan(None, src, leaf=0))
    bad = p.x.copy()
    bad[7] = np.nan
    _expect(_lib.EINVAL, lambda: api.HostPlan(None, (bad, p.y, p.z, p.q)))
    badq = p.q.copy()
    badq[3] = np.inf
    _expect(_lib.EINVAL, lambda: api.HostPlan(None, (p.x, p.y, p.z, badq)))
    with pytest.raises(ValueError):
        api.HostPlan(None, src, kernel="gravity")
    L = _lib.lib()
    # NULL handles and arrays through the raw ABI
    assert L.bldtt_setup_host(None, None, 0, 0.0, 0.7, 6, 10, 0) == _lib.EINVAL
    h = C.c_void_p()
    assert L.bldtt_setup_host(C.byref(h), None, 0, 0.0, 0.7, 6, 10, 0) == _lib.EINVAL and not h.value
    assert L.bldtt_destroy(None) == _lib.OK
    assert L.bldtt_compute(None, None, None) == _lib.EINVAL
    assert b"NULL" in L.bldtt_last_error()
    # the allocator hook takes both callbacks or neither
    cb = _lib.ALLOC_FN(lambda n, ctx: None)
    assert L.bldtt_set_allocator(C.cast(cb, C.c_void_p), None, None) == _lib.EINVAL
    assert b"both" in L.bldtt_last_error()
    api.use_torch_allocator()                       # the binding's registration, restored


def test_host_plan_refuses_compute_and_lists_before_traversal():
    p = inputs.particles(500, seed=36)
    hp = api.HostPlan(None, (p.x, p.y, p.z, p.q), theta=0.7, degree=2, leaf=50)
    _expect(_lib.ESTATE, hp.lists)
    L = _lib.lib()
    assert L.bldtt_compute(hp._handle, C.c_void_p(8), None) == _lib.ESTATE
    assert L.bldtt_get_qhat(hp._handle, (C.c_double * 8)()) == _lib.ESTATE


def test_interaction_counts_match_lists():
    p = inputs.particles(20_000, seed=37)
    hp = api.HostPlan(None, (p.x, p.y, p.z, p.q), theta=0.7, degree=4, leaf=200)
    hp.traverse_host()
    tree, L, st = hp.tree(0), hp.lists(), hp.stats()
    P = 125
    cnt = tree["count"]
    expect = {"PP": sum(cnt[t] * cnt[s] for t, s in zip(*L["PP"])),
              "PC": sum(cnt[t] * P for t in L["PC"][0]),
              "CP": sum(P * cnt[s] for s in L["CP"][1]),
              "CC": P * P * len(L["CC"][0])}
    for k in expect:
        assert st["interactions"][k] == expect[k]
    # pairs covered by PP alone would be N^2; the method evaluates far fewer kernels
    assert sum(st["interactions"].values()) < 0.5 * 20_000 ** 2
