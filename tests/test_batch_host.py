"""Host logic of the batched launch, on the CPU.

The forest of a batch is the concatenation of each problem's own trees (ids
shifted), and the dual tree traversal from every pair of roots (Algorithm 2)
gives each problem exactly its own lists; both are checked against the
oracle's tree build and traversal run on each problem alone."""
import numpy as np
import pytest

from oracle import core
from paper_2012_06925_amd import inputs

api = pytest.importorskip("paper_2012_06925_amd.api")
from paper_2012_06925_amd import _lib  # noqa: E402

TYPES = ("PP", "PC", "CP", "CC")


def _problems(count=7, seed=inputs.BASE_SEED + 40):
    # sizes 10^2.5 .. 10^3.6, distributions drawn per problem
    return inputs.batch_problems(count=count, seed=seed, lo_exp=2.5, hi_exp=3.6)


def _segment_matches(forest, local, c0, p0, caller0):
    nc = len(local["radius"])
    sl = slice(c0, c0 + nc)
    for k in ("lo", "hi", "center", "radius", "count", "level", "nchild"):
        assert np.array_equal(forest[k][sl], local[k]), k
    assert np.array_equal(forest["begin"][sl], local["begin"] + p0)
    shift = lambda a: np.where(a < 0, -1, a + c0)
    assert np.array_equal(forest["parent"][sl], shift(local["parent"]))
    assert np.array_equal(forest["child"][sl], shift(local["child"]))
    n = int(local["count"][0])
    assert np.array_equal(forest["perm"][p0:p0 + n], local["perm"] + caller0)
    return nc, n


def _check_lists(forest_lists, per_problem, offsets_t, offsets_s):
    for k in TYPES:
        tc, sc = forest_lists[k]
        got = sorted(zip(tc.tolist(), sc.tolist()))
        want = []
        for (lt, ls), ct, cs in zip(per_problem, offsets_t, offsets_s):
            want += [(int(a) + ct, int(b) + cs) for a, b in zip(*lt[k])] if lt[k][0].size else []
        assert got == sorted(want), k


@pytest.mark.parametrize("theta,deg,leaf", [(0.7, 6, 50), (0.9, 3, 20)])
def test_forest_and_lists_equal_per_problem_oracle_runs(theta, deg, leaf):
    probs = _problems()
    hb = api.HostBatch([(None, (p.x, p.y, p.z, p.q)) for _, p in probs], theta=theta, degree=deg, leaf=leaf)
    ft, fs = hb.tree(0), hb.tree(1)
    assert ft["radius"].size == fs["radius"].size        # targets = sources: one forest
    c0 = p0 = 0
    offs, per = [], []
    for _, p in probs:
        r = core.Run(p, p, theta=theta, degree=deg, leaf=leaf)
        r.traverse()
        nc, n = _segment_matches(fs, r.tree(1), c0, p0, p0)
        offs.append(c0)
        per.append(r.lists())
        c0 += nc
        p0 += n
    assert c0 == fs["radius"].size and p0 == fs["perm"].size
    _check_lists(hb.lists(), list(zip(per, per)), offs, offs)
    st = hb.stats()
    assert st["n_problems"] == len(probs)
    assert st["n_targets"] == sum(p.x.size for _, p in probs)
    assert st["n_tasks"] > 0
    hb.close()


def test_unequal_sets_forest():
    rng = np.random.default_rng(5)
    probs = _problems(count=4, seed=inputs.BASE_SEED + 41)
    batch, per, offs_t, offs_s = [], [], [], []
    ct = cs = pt = ps = 0
    pairs = []
    for i, (_, p) in enumerate(probs):
        if i % 2:
            t = rng.uniform(-0.5, 0.5, size=(3, 300 + 100 * i))
            batch.append(((t[0], t[1], t[2]), (p.x, p.y, p.z, p.q)))
            tgt = inputs.ParticleSet(t[0], t[1], t[2], np.zeros(t.shape[1]))
        else:
            batch.append((None, (p.x, p.y, p.z, p.q)))
            tgt = p
        pairs.append((tgt, p))
    hb = api.HostBatch(batch, theta=0.8, degree=4, leaf=40)
    ft, fs = hb.tree(0), hb.tree(1)
    for tgt, src in pairs:
        r = core.Run(tgt, src, theta=0.8, degree=4, leaf=40)
        r.traverse()
        nct, nt = _segment_matches(ft, r.tree(0), ct, pt, pt)
        ncs, ns = _segment_matches(fs, r.tree(1), cs, ps, ps)
        per.append(r.lists())
        offs_t.append(ct)
        offs_s.append(cs)
        ct, cs, pt, ps = ct + nct, cs + ncs, pt + nt, ps + ns
    _check_lists(hb.lists(), [(l, l) for l in per], offs_t, offs_s)
    hb.close()


def test_host_batch_refuses_device_calls_and_bad_arguments():
    probs = _problems(count=2)
    src = [(None, (p.x, p.y, p.z, p.q)) for _, p in probs]
    hb = api.HostBatch(src, theta=0.7, degree=6, leaf=50)
    assert hb.compute_raw() == _lib.ESTATE
    hb.close()
    with pytest.raises(_lib.BldttError) as e:
        api.HostBatch(src, degree=6, leaf=50, flags=_lib.LEARNED_DEGREE)
    assert e.value.code == _lib.EUNSUPPORTED
    with pytest.raises(_lib.BldttError) as e:
        api.HostBatch(src, degree=6, leaf=50, tpt=3)
    assert e.value.code == _lib.EINVAL
    with pytest.raises(_lib.BldttError) as e:
        api.HostBatch(src, theta=1.5)
    assert e.value.code == _lib.EINVAL
    with pytest.raises(_lib.BldttError) as e:
        api.HostBatch([], theta=0.7)
    assert e.value.code == _lib.EINVAL
