"""bldtt_set_allocator through the C ABI: plans and batches take their device
memory from the registered allocator and give all of it back; an allocator
that returns NULL makes the call fail with BLDTT_ENOMEM, every buffer
allocated before the failure released (counted in the callbacks)."""
import gc

import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import core  # noqa: E402
from paper_2012_06925_amd import inputs  # noqa: E402


def _api():
    from paper_2012_06925_amd import api
    return api


class Counting:
    """Device memory from torch's caching allocator, counted; NULL after `fail_after` allocations."""

    def __init__(self, fail_after=None):
        self.fail_after = fail_after
        self.live = {}
        self.n_alloc = self.n_release = self.n_refused = 0

    def alloc(self, n):
        if self.fail_after is not None and self.n_alloc >= self.fail_after:
            self.n_refused += 1
            return 0
        p = torch.cuda.caching_allocator_alloc(n)
        self.live[p] = n
        self.n_alloc += 1
        return p

    def release(self, p):
        assert p in self.live, "released a pointer the allocator did not hand out"
        del self.live[p]
        self.n_release += 1
        torch.cuda.caching_allocator_delete(p)


def _src(n, seed):
    p = inputs.particles(n, "uniform", seed=seed)
    return p, [torch.from_numpy(a).cuda() for a in (p.x, p.y, p.z, p.q)]


def test_plan_memory_comes_from_the_registered_allocator():
    api = _api()
    p, src = _src(20_000, 90)
    cnt = Counting()
    api.set_allocator(cnt.alloc, cnt.release)
    try:
        plan = api.Plan(None, src, theta=0.7, degree=5, leaf=200)
        phi = plan.compute().cpu().numpy()
        phi2 = plan.compute().cpu().numpy()
        assert cnt.n_alloc > 10 and cnt.live
        plan.close()
        assert not cnt.live and cnt.n_release == cnt.n_alloc
    finally:
        api.use_torch_allocator()
    ref = core.bldtt(p, p, theta=0.7, degree=5, leaf=200)
    for got in (phi, phi2):
        assert core.rel_l2(got, ref) < 1e-12 and core.max_rel(got, ref) < 1e-12


def test_failing_allocator_gives_enomem_and_releases_everything():
    # count the allocations of a full setup, then refuse the first, the
    # second, one in the middle and the last of them
    api = _api()
    from paper_2012_06925_amd import _lib
    _, src = _src(30_000, 91)
    flags = _lib.FP32_EVAL | _lib.LEARNED_DEGREE
    kw = dict(theta=0.7, degree=5, leaf=200, flags=flags)
    probe = Counting()
    api.set_allocator(probe.alloc, probe.release)
    try:
        api.Plan(None, src, **kw).close()
    finally:
        api.use_torch_allocator()
    n = probe.n_alloc
    assert n > 8 and not probe.live
    for fail_after in sorted({0, 1, n // 2, n - 1}):
        gc.collect()
        torch.cuda.synchronize()
        base = torch.cuda.memory_allocated()
        cnt = Counting(fail_after)
        api.set_allocator(cnt.alloc, cnt.release)
        try:
            with pytest.raises(_lib.BldttError) as e:
                api.Plan(None, src, **kw)
        finally:
            api.use_torch_allocator()
        assert e.value.code == _lib.ENOMEM, e.value
        assert cnt.n_refused == 1 and cnt.n_alloc == fail_after, (fail_after, cnt.n_refused, cnt.n_alloc)
        assert not cnt.live and cnt.n_release == cnt.n_alloc
        torch.cuda.synchronize()
        assert torch.cuda.memory_allocated() <= base          # nothing the failed call took is still held


def test_failing_allocator_during_compute_and_batch_setup():
    # a plan set up normally whose allocator then refuses: the compute that
    # needs new buffers fails with ENOMEM, and destroying the plan releases all
    api = _api()
    from paper_2012_06925_amd import _lib
    _, src = _src(30_000, 92)
    cnt = Counting()
    api.set_allocator(cnt.alloc, cnt.release)
    try:
        plan = api.Plan(None, src, theta=0.7, degree=5, leaf=200)
        cnt.fail_after = cnt.n_alloc          # setup done: refuse every later request
        with pytest.raises(_lib.BldttError) as e:
            plan.compute()
        assert e.value.code == _lib.ENOMEM
        plan.close()
        assert not cnt.live and cnt.n_release == cnt.n_alloc
        # a batch whose setup runs out part way
        probs = [(None, tuple(torch.from_numpy(a).cuda() for a in (q.x, q.y, q.z, q.q)))
                 for _, q in inputs.batch_problems(count=6, seed=93, lo_exp=2.5, hi_exp=3.5)]
        cnt2 = Counting(fail_after=12)
        api.set_allocator(cnt2.alloc, cnt2.release)
        with pytest.raises(_lib.BldttError) as e:
            api.Batch(probs, theta=0.7, degree=5, leaf=60)
        assert e.value.code == _lib.ENOMEM
        assert not cnt2.live and cnt2.n_release == cnt2.n_alloc == 12
    finally:
        api.use_torch_allocator()
