"""The list-building walk on the GPU (BLDTT_DEVICE_TRAVERSAL) against the
oracle's walks and the library's host walk: MAC ties (theta equal to the
exact ratio of a pair the walk meets, and one ulp above it), every scheme,
the per-pair degree deferral, the same lists as the host walk and potentials
equal to rounding, and bit-identical recomputes."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import core  # noqa: E402
from paper_2012_06925_amd import inputs  # noqa: E402

DEVICE_TRAVERSAL = 2048
SCHEME_FLAGS = {"bldtt": 0, "pp_cc_only": 16, "bltc": 512, "cp_bltc": 1024}


def _api():
    from paper_2012_06925_amd import api
    return api


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _sets(L):
    return {k: sorted(zip(L[k][0].tolist(), L[k][1].tolist())) for k in ("PP", "PC", "CP", "CC")}


def _plan_lists(tgt, src, same, theta, degree, leaf, flags):
    api = _api()
    s = [dev(a) for a in (src.x, src.y, src.z, src.q)]
    t = None if same else [dev(a) for a in (tgt.x, tgt.y, tgt.z)]
    plan = api.Plan(t, s, theta=theta, degree=degree, leaf=leaf, flags=flags)
    phi = plan.compute().cpu().numpy()
    L = plan.lists()
    st = plan.stats()
    plan.close()
    return phi, L, st


def _mac_ratio(tt, ts, t, s):
    # the MAC's left side in the order every walk evaluates it
    d = tt["center"][t] - ts["center"][s]
    R = np.sqrt((d[0] * d[0] + d[1] * d[1]) + d[2] * d[2])
    return (tt["radius"][t] + ts["radius"][s]) / R


@pytest.mark.parametrize("case", ["same", "unequal"])
def test_mac_ties_give_the_oracle_lists(case):
    # theta = the exact ratio of a separated pair: that pair is no longer
    # separated (strict '<'); one ulp above, it is again.  A rounding
    # difference anywhere in R, the radii sum or the division moves entries.
    if case == "same":
        t = s = inputs.particles(20_000, "gaussian", seed=inputs.BASE_SEED + 330)
    else:
        t, s = inputs.unequal_sets(15_000, "sphere", 20_000, "uniform", seed=inputs.BASE_SEED + 331)
    base = core.Run(t, s, theta=0.7, degree=3, leaf=40, aliased=case == "same")
    base.traverse()
    tt, ts = base.tree(0), base.tree(1)
    L = base.lists()
    rng = np.random.default_rng(7)
    picks = []
    for k in ("CC", "PC", "CP"):
        if len(L[k][0]):
            for e in rng.choice(len(L[k][0]), size=min(2, len(L[k][0])), replace=False):
                picks.append(_mac_ratio(tt, ts, L[k][0][e], L[k][1][e]))
    assert len(picks) >= 4
    for ratio in picks:
        for theta in (float(ratio), float(np.nextafter(ratio, 1.0))):
            ref = core.Run(t, s, theta=theta, degree=3, leaf=40, aliased=case == "same")
            ref.traverse()
            _, got, _ = _plan_lists(t, s, case == "same", theta, 3, 40, DEVICE_TRAVERSAL)
            assert _sets(got) == _sets(ref.lists()), (ratio, theta)


@pytest.mark.parametrize("scheme", sorted(SCHEME_FLAGS))
def test_device_and_host_walks_agree(scheme):
    # same lists as sets, same interaction counts, potentials equal to rounding,
    # and both equal to the oracle's lists
    p = inputs.particles(60_000, "plummer", seed=inputs.BASE_SEED + 332)
    fl = SCHEME_FLAGS[scheme]
    phi_d, Ld, std = _plan_lists(p, p, True, 0.75, 4, 150, fl | DEVICE_TRAVERSAL)
    phi_h, Lh, sth = _plan_lists(p, p, True, 0.75, 4, 150, fl)
    assert _sets(Ld) == _sets(Lh)
    assert std["interactions"] == sth["interactions"]
    assert core.max_rel(phi_d, phi_h) < 1e-14
    ref = core.Run(p, p, theta=0.75, degree=4, leaf=150, scheme=scheme)
    ref.traverse()
    assert _sets(Ld) == _sets(ref.lists())


def test_device_walk_recompute_is_bit_identical_with_one_sided_passes():
    # the device walk is deterministic: with one-sided passes (no atomics) two
    # computes give the same bits
    p = inputs.particles(40_000, "uniform", seed=inputs.BASE_SEED + 333)
    api = _api()
    s = [dev(a) for a in (p.x, p.y, p.z, p.q)]
    plan = api.Plan(None, s, theta=0.8, degree=5, leaf=200, flags=256 | DEVICE_TRAVERSAL)
    a = plan.compute().cpu().numpy()
    b = plan.compute().cpu().numpy()
    L1 = plan.lists()
    c = plan.compute().cpu().numpy()
    L2 = plan.lists()
    plan.close()
    assert np.array_equal(a, b) and np.array_equal(b, c)
    for k in L1:
        assert np.array_equal(L1[k][0], L2[k][0]) and np.array_equal(L1[k][1], L2[k][1])
