"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Each test names what it pins.  None of them re-types the oracle's own formula:
the checks use closed forms, hand-worked values, identities of polynomial
interpolation (Appendix A), independent brute-force forms (product-form
Lagrange polynomials and explicit approximated-kernel matrices), invariants of
the tree and of the traversal, and the paper's own error table.
"""
import json
import math
import os

import numpy as np
import pytest

from oracle import brute, core
from paper_2012_06925_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _xyz(p):
    return p.xyz()


# --------------------------------------------------------------------------
# Direct sum, Eq. (1)
# --------------------------------------------------------------------------

def test_direct_sum_two_particles_hand_values():
    # phi = q / r for Coulomb and q e^{-kappa r} / r for Yukawa; the self term is skipped.
    t = inputs.ParticleSet(np.array([0.0, 3.0]), np.array([0.0, 4.0]), np.array([0.0, 0.0]), np.array([2.0, -1.0]))
    phi = core.direct_sum(t, t)
    assert phi[0] == pytest.approx(-1.0 / 5.0, rel=1e-15)
    assert phi[1] == pytest.approx(2.0 / 5.0, rel=1e-15)
    phy = core.direct_sum(t, t, kernel="yukawa")
    assert phy[0] == pytest.approx(-math.exp(-2.5) / 5.0, rel=1e-14)
    assert phy[1] == pytest.approx(2.0 * math.exp(-2.5) / 5.0, rel=1e-14)


def _pair(dist, q=1.0):
    t = inputs.ParticleSet(np.array([0.0]), np.array([0.0]), np.array([0.0]), np.array([1.0]))
    s = inputs.ParticleSet(np.array([dist]), np.array([0.0]), np.array([0.0]), np.array([q]))
    return t, s


@pytest.mark.parametrize("r,value", [(0.5, 2.0), (1.0 / 6.0, 3.0), (1.5, -2.0 / 3.0)])
def test_oscillatory_kernel_hand_values(r, value):
    # Sec. 4.6 oscillatory kernel sin(pi r)/r: sin(pi/2)/(1/2) = 2,
    # sin(pi/6)/(1/6) = 3, sin(3 pi/2)/(3/2) = -2/3
    t, s = _pair(r)
    assert core.direct_sum(t, s, kernel="oscillatory")[0] == pytest.approx(value, rel=1e-14)
    assert brute.direct_sum(t.xyz(), s.xyz(), s.q, "oscillatory")[0] == pytest.approx(value, rel=1e-14)
    # the whole method with one leaf (a single PP pair) gives the same value
    assert core.bldtt(t, s, kernel="oscillatory", theta=0.5, degree=2, leaf=4)[0] == pytest.approx(value, rel=1e-14)


@pytest.mark.parametrize("r,eps,value", [(0.012, 0.005, 1.0 / 0.013), (4.0, 3.0, 0.2), (0.0048, 0.0014, 200.0)])
def test_regularized_coulomb_hand_values(r, eps, value):
    # Sec. 4.6 regularized Coulomb 1/sqrt(r^2 + eps^2), eps = 0.005 in the
    # paper: (12, 5, 13) and (4, 3, 5) and (48, 14, 50) right triangles
    t, s = _pair(r)
    assert core.direct_sum(t, s, kernel="regcoulomb", param=eps)[0] == pytest.approx(value, rel=1e-14)
    assert brute.direct_sum(t.xyz(), s.xyz(), s.q, "regcoulomb", eps)[0] == pytest.approx(value, rel=1e-14)
    got = core.bldtt(t, s, kernel="regcoulomb", param=eps, theta=0.5, degree=2, leaf=4)[0]
    assert got == pytest.approx(value, rel=1e-14)


def test_regularized_coulomb_default_eps_is_paper_value():
    # the paper's eps = 0.005: at r = 0.012 the kernel is 1/0.013, not 1/0.012
    t, s = _pair(0.012)
    assert core.DEFAULT_PARAM["regcoulomb"] == 0.005
    assert core.direct_sum(t, s, kernel="regcoulomb")[0] == pytest.approx(1.0 / 0.013, rel=1e-14)


def test_direct_sum_matches_numpy_matrix_form():
    t, s = inputs.unequal_sets(300, "sphere", 500, "gaussian", seed=7)
    for kernel, param in (("coulomb", 0.0), ("yukawa", 0.5), ("oscillatory", 0.0), ("regcoulomb", 0.005)):
        ref = brute.direct_sum(_xyz(t), _xyz(s), s.q, kernel, param)
        got = core.direct_sum(t, s, kernel=kernel, param=param)
        assert core.rel_l2(got, ref) < 1e-13, kernel


def test_direct_sum_compensated_is_exact_on_cancelling_terms():
    # charges +1e16, 1, -1e16 at equal distance: a naive left-to-right sum loses the 1.
    tx = np.array([0.0])
    t = inputs.ParticleSet(tx, tx.copy(), tx.copy())
    s = inputs.ParticleSet(np.array([1.0, 0.0, 0.0]), np.array([0.0, 1.0, 0.0]), np.array([0.0, 0.0, 1.0]),
                           np.array([1e16, 1.0, -1e16]))
    assert core.direct_sum(t, s)[0] == 1.0


def test_direct_sum_selection_equals_full():
    p = inputs.particles(800, seed=3)
    full = core.direct_sum(p, p)
    sel = np.array([5, 17, 799, 0])
    assert np.array_equal(core.direct_sum(p, p, sel=sel), full[sel])


# --------------------------------------------------------------------------
# Chebyshev points and weights (Sec. 2.1), barycentric basis (Eq. 2)
# --------------------------------------------------------------------------

def test_cheb_hand_values():
    g = json.load(open(os.path.join(GOLDEN, "cheb_n2.json")))
    for key, n in (("n2", 2), ("n3", 3)):
        xi, w = core.cheb(n)
        np.testing.assert_allclose(xi, g[key]["xi"], rtol=0, atol=2.3e-16)
        assert list(w) == g[key]["w"]


@pytest.mark.parametrize("n", [1, 2, 3, 5, 8, 12])
def test_cheb_nodes_and_weights(n):
    xi, w = core.cheb(n)
    assert xi[0] == 1.0 and xi[n] == -1.0
    assert np.array_equal(xi[::-1], -xi)                       # exactly antisymmetric
    np.testing.assert_allclose(xi, np.cos(np.pi * np.arange(n + 1) / n), rtol=0, atol=4.5e-16)
    # The closed-form weights are proportional to the general definition of Eq. (2).
    g = brute.general_weights(brute.cheb_points(n))
    np.testing.assert_allclose(w / w[0], g / g[0], rtol=1e-12)


@pytest.mark.parametrize("n", [1, 2, 4, 7, 10, 12])
def test_basis_kronecker_at_nodes(n):
    lo, hi = -0.3, 1.7
    xi, _ = core.cheb(n)
    s = 0.5 * (lo + hi) + 0.5 * (hi - lo) * xi
    for j in range(n + 1):
        L = core.basis1d(n, lo, hi, s[j])
        e = np.zeros(n + 1)
        e[j] = 1.0
        assert np.array_equal(L, e)


@pytest.mark.parametrize("n", [1, 3, 6, 9, 12])
def test_basis_vs_product_form_and_partition_of_unity(n):
    rng = np.random.default_rng(n)
    lo, hi = -1.2, 0.4
    for y in rng.uniform(lo, hi, size=40):
        L = core.basis1d(n, lo, hi, y)
        ref = brute.lagrange_product(brute.box_points(n, lo, hi), np.array([y]))[0]
        np.testing.assert_allclose(L, ref, rtol=0, atol=1e-13)
        assert abs(L.sum() - 1.0) < 1e-14 * max(1.0, np.abs(L).sum())


@pytest.mark.parametrize("n", [2, 5, 8])
def test_basis_reproduces_polynomials_up_to_degree_n(n):
    # Appendix A: the degree-n interpolant of a degree <= n polynomial is itself.
    lo, hi = 0.25, 2.0
    xi, _ = core.cheb(n)
    s = 0.5 * (lo + hi) + 0.5 * (hi - lo) * xi
    ys = np.linspace(lo, hi, 17) + 1e-3
    for deg in range(n + 1):
        for y in ys:
            L = core.basis1d(n, lo, hi, y)
            assert abs(L @ s ** deg - y ** deg) < 1e-12 * max(1.0, y ** deg)
    # degree n+1 is not reproduced (sanity: the test can fail)
    errs = [abs(core.basis1d(n, lo, hi, y) @ s ** (n + 1) - y ** (n + 1)) for y in ys]
    assert max(errs) > 1e-6


def test_basis_flat_box():
    # zero-width box: every node equals the point, node 0 carries everything
    L = core.basis1d(4, 0.5, 0.5, 0.5)
    assert list(L) == [1.0, 0.0, 0.0, 0.0, 0.0]


# --------------------------------------------------------------------------
# Trees (Sec. 2.3)
# --------------------------------------------------------------------------

def _check_tree_invariants(tree, xyz, leaf):
    nc = tree["lo"].shape[0]
    perm = tree["perm"]
    assert np.array_equal(np.sort(perm), np.arange(xyz.shape[0]))
    for c in range(nc):
        b, cnt = tree["begin"][c], tree["count"][c]
        pts = xyz[perm[b:b + cnt]]
        # minimal box
        assert np.array_equal(pts.min(axis=0), tree["lo"][c])
        assert np.array_equal(pts.max(axis=0), tree["hi"][c])
        nk = tree["nchild"][c]
        L = tree["hi"][c] - tree["lo"][c]
        if nk == 0:
            continue
        assert cnt > leaf and L.max() > 0.0
        kids = tree["child"][c][:nk]
        # children partition the parent's range, in order, and point back to it
        pos = b
        for k in kids:
            assert tree["begin"][k] == pos and tree["parent"][k] == c
            assert tree["level"][k] == tree["level"][c] + 1
            pos += tree["count"][k]
        assert pos == b + cnt
        # number of split dimensions obeys the count caps, and at most 2^dims children
        cap = 1 if cnt <= 2 * leaf else (2 if cnt <= 4 * leaf else 3)
        assert nk <= 2 ** cap
        # DFS preorder: first child follows its parent immediately
        assert kids[0] == c + 1


@pytest.mark.parametrize("dist,n,leaf", [("uniform", 5000, 100), ("gaussian", 4000, 50), ("sphere", 3000, 64),
                                         ("rod", 2000, 30), ("slab", 2000, 30)])
def test_tree_invariants_random(dist, n, leaf):
    p = inputs.particles(n, dist, seed=11)
    tree = core.build_tree(p, leaf)
    _check_tree_invariants(tree, p.xyz(), leaf)
    leaves = tree["nchild"] == 0
    # every leaf within the size limit (no degenerate boxes here)
    assert tree["count"][leaves].max() <= leaf


def test_tree_cube_corners_eight_leaves():
    c = np.array([[x, y, z] for z in (0.0, 1.0) for y in (0.0, 1.0) for x in (0.0, 1.0)])
    p = inputs.ParticleSet(*[c[:, d].copy() for d in range(3)])
    tree = core.build_tree(p, 1)
    assert tree["lo"].shape[0] == 9 and tree["nchild"][0] == 8
    # child code x + 2y + 4z; preorder numbering gives corner k at cluster k + 1
    for k in range(8):
        assert tree["perm"][tree["begin"][k + 1]] == k


def test_tree_coplanar_points_split_four_ways():
    rng = np.random.default_rng(2)
    n = 4000
    p = inputs.ParticleSet(rng.uniform(-1, 1, n), rng.uniform(-1, 1, n), np.zeros(n))
    tree = core.build_tree(p, 100)
    internal = tree["nchild"] > 0
    assert tree["nchild"][internal].max() == 4
    _check_tree_invariants(tree, p.xyz(), 100)


def test_tree_collinear_points_split_two_ways():
    rng = np.random.default_rng(3)
    n = 3000
    p = inputs.ParticleSet(rng.uniform(-1, 1, n), np.full(n, 0.5), np.full(n, -0.25))
    tree = core.build_tree(p, 100)
    internal = tree["nchild"] > 0
    assert tree["nchild"][internal].max() == 2
    _check_tree_invariants(tree, p.xyz(), 100)


def test_tree_identical_points_single_guarded_leaf():
    n = 50
    p = inputs.ParticleSet(np.full(n, 0.1), np.full(n, 0.2), np.full(n, 0.3))
    tree = core.build_tree(p, 4)
    assert tree["lo"].shape[0] == 1 and tree["nchild"][0] == 0 and tree["count"][0] == n


def test_tree_aspect_rule_long_box():
    # points on a 1 x 1 x 4 box: only z qualifies (2*1 < 16), so the first split is two-way in z
    rng = np.random.default_rng(4)
    n = 20000
    p = inputs.ParticleSet(rng.uniform(0, 1, n), rng.uniform(0, 1, n), rng.uniform(0, 4, n))
    tree = core.build_tree(p, 100)
    assert tree["nchild"][0] == 2
    k0 = tree["child"][0][0]
    assert tree["hi"][k0][2] < 2.0 + 1e-9 and tree["hi"][k0][0] > 0.9


def test_tree_aspect_rule_sqrt2_threshold():
    # box 1 x 1.3 x 1.6: Lmax^2 = 2.56; y qualifies (2*1.69 >= 2.56), x does not (2*1 < 2.56),
    # so a cluster with more than 4 leaves' worth of points splits in y and z only: 4 children.
    rng = np.random.default_rng(5)
    n = 20000
    xyz = rng.uniform(0, 1, (n, 3)) * np.array([1.0, 1.3, 1.6])
    xyz[0] = [0.0, 0.0, 0.0]
    xyz[1] = [1.0, 1.3, 1.6]
    p = inputs.ParticleSet(*[xyz[:, d].copy() for d in range(3)])
    tree = core.build_tree(p, 100)
    assert tree["nchild"][0] == 4
    kids = tree["child"][0][:4]
    # children split at y = 0.65 and z = 0.8; none is cut in x
    for k in kids:
        assert tree["hi"][k][0] - tree["lo"][k][0] > 0.99


# --------------------------------------------------------------------------
# Dual tree traversal, Algorithm 2
# --------------------------------------------------------------------------

def test_traversal_tie_descends_into_source_hand_case():
    # |C_t| == |C_s| == 2, roots not separated: Algorithm 2 descends into the source.
    # T = {(0,0,0), (1,0,0)} (r_t = 0.5); S = {(20,0,0), (1.2,0,0)} (box [1.2, 20], r_s = 9.4).
    # Source children: s(1.2) -> cluster 1, s(20) -> cluster 2.  Target children t(0) -> 1, t(1) -> 2.
    #   DTT(T, s@1.2): R = 0.7, 0.5/0.7 > 0.7 -> not separated, s leaf -> children of T:
    #       (1, 1) and (2, 1) separated with zero radii -> PP
    #   DTT(T, s@20): R = 19.5 -> separated, both small -> PP (0, 2)
    t = inputs.ParticleSet(np.array([0.0, 1.0]), np.zeros(2), np.zeros(2))
    s = inputs.ParticleSet(np.array([20.0, 1.2]), np.zeros(2), np.zeros(2), np.ones(2))
    run = core.Run(t, s, theta=0.7, degree=1, leaf=1)
    run.traverse()
    L = run.lists()
    assert set(zip(*L["PP"])) == {(1, 1), (2, 1), (0, 2)}
    assert all(len(L[k][0]) == 0 for k in ("PC", "CP", "CC"))

def _coverage(run, M, N):
    """Count how often each (target, source) pair is covered by a list entry."""
    tt, ts = run.tree(0), run.tree(1)
    cover = np.zeros((M, N), dtype=np.int32)
    for name, (tcs, scs) in run.lists().items():
        for tc, sc in zip(tcs, scs):
            ti = tt["perm"][tt["begin"][tc]:tt["begin"][tc] + tt["count"][tc]]
            sj = ts["perm"][ts["begin"][sc]:ts["begin"][sc] + ts["count"][sc]]
            cover[np.ix_(ti, sj)] += 1
    return cover


@pytest.mark.parametrize("case", ["same", "unequal"])
@pytest.mark.parametrize("theta,n,leaf", [(0.5, 1, 20), (0.7, 2, 40), (0.9, 1, 8)])
def test_lists_cover_every_pair_once(case, theta, n, leaf):
    if case == "same":
        t = s = inputs.particles(1500, "gaussian", seed=5)
    else:
        t, s = inputs.unequal_sets(900, "sphere", 1400, "uniform", seed=6)
    run = core.Run(t, s, theta=theta, degree=n, leaf=leaf)
    run.traverse()
    cover = _coverage(run, t.n, s.n)
    assert cover.min() == 1 and cover.max() == 1


@pytest.mark.parametrize("theta,n", [(0.5, 1), (0.7, 2), (0.9, 1)])
def test_lists_mac_and_types(theta, n):
    t, s = inputs.unequal_sets(3000, "uniform", 2500, "gaussian", seed=8)
    run = core.Run(t, s, theta=theta, degree=n, leaf=20)
    run.traverse()
    tt, ts = run.tree(0), run.tree(1)
    npx = (n + 1) ** 3
    for name, (tcs, scs) in run.lists().items():
        for tc, sc in zip(tcs, scs):
            R = np.linalg.norm(tt["center"][tc] - ts["center"][sc])
            sep = R > 0 and (tt["radius"][tc] + ts["radius"][sc]) / R < theta
            big_t, big_s = tt["count"][tc] > npx, ts["count"][sc] > npx
            if name == "CC":
                assert sep and big_t and big_s
            elif name == "CP":
                assert sep and big_t and not big_s
            elif name == "PC":
                assert sep and not big_t and big_s
            else:
                leaves = tt["nchild"][tc] == 0 and ts["nchild"][sc] == 0
                assert (sep and not big_t and not big_s) or (not sep and leaves)
    counts = {k: len(v[0]) for k, v in run.lists().items()}
    assert counts["CC"] > 0 and counts["PP"] > 0


def _ablation_runs(case, theta, n, leaf):
    if case == "same":
        t = s = inputs.particles(1500, "gaussian", seed=25)
    else:
        t, s = inputs.unequal_sets(900, "sphere", 1400, "uniform", seed=26)
    full = core.Run(t, s, theta=theta, degree=n, leaf=leaf)
    abl = core.Run(t, s, theta=theta, degree=n, leaf=leaf, pp_cc_only=True)
    full.traverse()
    abl.traverse()
    return t, s, full, abl


@pytest.mark.parametrize("case", ["same", "unequal"])
@pytest.mark.parametrize("theta,n,leaf", [(0.7, 1, 10), (0.9, 2, 8)])
def test_ablation_lists_cover_every_pair_once_and_keep_the_recursion(case, theta, n, leaf):
    # Sec. 4.3 ablation (CC and PP only): the recursion of Algorithm 2 is the
    # same, so the separated pairs are the same; a pair is CC when both
    # clusters hold more than (n+1)^3 particles and PP otherwise.  Hence:
    # every (i, j) covered once, no PC/CP, CC equal to the full traversal's
    # CC, and PP = full PP + PC + CP.
    t, s, full, abl = _ablation_runs(case, theta, n, leaf)
    A, F = abl.lists(), full.lists()
    cover = _coverage(abl, t.n, s.n)
    assert cover.min() == 1 and cover.max() == 1
    assert len(A["PC"][0]) == 0 and len(A["CP"][0]) == 0
    assert len(F["PC"][0]) > 0 and len(F["CP"][0]) > 0 and len(F["CC"][0]) > 0
    pairs = lambda L, k: set(zip(L[k][0].tolist(), L[k][1].tolist()))
    assert pairs(A, "CC") == pairs(F, "CC")
    assert pairs(A, "PP") == pairs(F, "PP") | pairs(F, "PC") | pairs(F, "CP")
    assert len(A["PP"][0]) == len(pairs(A, "PP"))
    tt, ts = abl.tree(0), abl.tree(1)
    npx = (n + 1) ** 3
    for tc, sc in zip(*A["CC"]):
        assert tt["count"][tc] > npx and ts["count"][sc] > npx
    for tc, sc in zip(*A["PP"]):
        R = np.linalg.norm(tt["center"][tc] - ts["center"][sc])
        sep = R > 0 and (tt["radius"][tc] + ts["radius"][sc]) / R < theta
        leaves = tt["nchild"][tc] == 0 and ts["nchild"][sc] == 0
        assert (sep and not (tt["count"][tc] > npx and ts["count"][sc] > npx)) or (not sep and leaves)


@pytest.mark.parametrize("case", ["same", "unequal"])
def test_ablation_potentials_equal_explicit_matrices(case):
    # the ablation's potentials are the sum of exact PP blocks and CC
    # interpolated blocks over its lists (explicit matrices, no up/down passes)
    n = 2
    t, s, full, abl = _ablation_runs(case, 0.9, n, 8)
    phi = abl.run_all()
    ref = brute.explicit_bldtt(t.xyz(), s.xyz(), s.q, abl.tree(0), abl.tree(1), abl.lists(), n)
    assert core.rel_l2(phi, ref) < 1e-13
    # and it differs from the four-type method only at the approximation level
    assert 0 < core.rel_l2(phi, full.run_all()) < 1e-2


# The two treecodes the paper compares with.  BLTC (Sec. 2.8): every target
# batch (a target leaf) walks the source tree; CP-BLTC (Sec. 4.5): every source
# batch (a source leaf) walks the target tree.  The walks are pinned against
# their characterisation, written without a walk: batch b meets cluster c of
# the walked tree iff no proper ancestor of c is separated from b; c is then a
# list entry iff it is separated from b or a leaf, by proxies iff separated
# and holding more than (n+1)^3 particles.

def _treecode_sets(case, seed):
    if case == "same":
        t = s = inputs.particles(1500, "gaussian", seed=seed)
    else:
        t, s = inputs.unequal_sets(900, "sphere", 1400, "uniform", seed=seed + 1)
    return t, s


def _sep(ta, a, tb, b, theta):
    R = np.linalg.norm(ta["center"][a] - tb["center"][b])
    return R > 0 and (ta["radius"][a] + tb["radius"][b]) / R < theta


def _ancestors(tree, c):
    out = []
    while tree["parent"][c] >= 0:
        c = int(tree["parent"][c])
        out.append(c)
    return out


def _treecode_lists_by_characterisation(tt, ts, theta, n, scheme):
    npx = (n + 1) ** 3
    batches, walked = (tt, ts) if scheme == "bltc" else (ts, tt)
    out = {k: set() for k in ("PP", "PC", "CP", "CC")}
    anc = [_ancestors(walked, c) for c in range(len(walked["count"]))]
    for b in np.flatnonzero(batches["nchild"] == 0):
        for c in range(len(walked["count"])):
            sep = (lambda x: _sep(tt, b, ts, x, theta)) if scheme == "bltc" else (lambda x: _sep(tt, x, ts, b, theta))
            if any(sep(a) for a in anc[c]):
                continue                                  # the walk stopped above c
            here = sep(c)
            if not here and walked["nchild"][c] != 0:
                continue                                  # passed on to the children
            kind = ("PC" if scheme == "bltc" else "CP") if here and walked["count"][c] > npx else "PP"
            out[kind].add((int(b), c) if scheme == "bltc" else (c, int(b)))
    return out


@pytest.mark.parametrize("scheme", ["bltc", "cp_bltc"])
@pytest.mark.parametrize("case", ["same", "unequal"])
@pytest.mark.parametrize("theta,n,leaf", [(0.5, 1, 20), (0.7, 1, 10), (0.9, 2, 8)])
def test_treecode_lists_equal_their_characterisation(scheme, case, theta, n, leaf):
    t, s = _treecode_sets(case, 61)
    run = core.Run(t, s, theta=theta, degree=n, leaf=leaf, scheme=scheme)
    run.traverse()
    L = run.lists()
    got = {k: set(zip(L[k][0].tolist(), L[k][1].tolist())) for k in L}
    assert all(len(got[k]) == len(L[k][0]) for k in L)            # no entry twice
    want = _treecode_lists_by_characterisation(run.tree(0), run.tree(1), theta, n, scheme)
    assert got == want
    approx = "PC" if scheme == "bltc" else "CP"
    assert len(got[approx]) > 0 and len(got["PP"]) > 0
    cover = _coverage(run, t.n, s.n)
    assert cover.min() == 1 and cover.max() == 1


@pytest.mark.parametrize("scheme", ["bltc", "cp_bltc"])
def test_treecode_types_and_batches(scheme):
    t, s = inputs.unequal_sets(3000, "uniform", 2500, "gaussian", seed=63)
    theta, n = 0.7, 1
    run = core.Run(t, s, theta=theta, degree=n, leaf=20, scheme=scheme)
    run.traverse()
    L = run.lists()
    tt, ts = run.tree(0), run.tree(1)
    npx = (n + 1) ** 3
    forbidden = ("CP", "CC") if scheme == "bltc" else ("PC", "CC")
    assert all(len(L[k][0]) == 0 for k in forbidden)
    batch, batch_tree, walked_tree = (0, tt, ts) if scheme == "bltc" else (1, ts, tt)
    approx = "PC" if scheme == "bltc" else "CP"
    for name in ("PP", approx):
        for tc, sc in zip(*L[name]):
            b, c = (tc, sc) if scheme == "bltc" else (sc, tc)
            assert batch_tree["nchild"][b] == 0                 # the batches are leaves
            sep = _sep(tt, tc, ts, sc, theta)
            if name == approx:
                assert sep and walked_tree["count"][c] > npx
            else:
                assert (sep and walked_tree["count"][c] <= npx) or (not sep and walked_tree["nchild"][c] == 0)
    # every batch starts at the root of the walked tree, so each batch has entries
    batches = set(np.flatnonzero(batch_tree["nchild"] == 0).tolist())
    seen = {int(e[batch]) for name in ("PP", approx) for e in zip(*L[name])}
    assert seen == batches


@pytest.mark.parametrize("scheme", ["bltc", "cp_bltc"])
@pytest.mark.parametrize("kernel", ["coulomb", "yukawa"])
@pytest.mark.parametrize("case", ["same", "unequal"])
def test_treecode_potentials_equal_explicit_matrices(scheme, kernel, case):
    # the upward pass (BLTC) or downward pass (CP-BLTC) of the oracle against the
    # approximated kernel written as explicit matrices per list entry
    n = 2
    t, s = _treecode_sets(case, 65)
    run = core.Run(t, s, kernel=kernel, theta=0.9, degree=n, leaf=8, scheme=scheme)
    phi = run.run_all()
    L = run.lists()
    assert len(L["PC" if scheme == "bltc" else "CP"][0]) > 0
    ref = brute.explicit_bldtt(t.xyz(), s.xyz(), s.q, run.tree(0), run.tree(1), L, n, kernel,
                               core.DEFAULT_PARAM[kernel])
    assert core.rel_l2(phi, ref) < 1e-13 and core.max_rel(phi, ref) < 1e-13


@pytest.mark.parametrize("scheme", ["bltc", "cp_bltc"])
def test_treecode_polynomial_kernel_is_reproduced_exactly(scheme):
    t, s = inputs.unequal_sets(2500, "uniform", 3000, "gaussian", seed=16)
    run = core.Run(t, s, kernel="poly", theta=0.7, degree=2, leaf=40, scheme=scheme)
    phi = run.run_all()
    assert len(run.lists()["PC" if scheme == "bltc" else "CP"][0]) > 0
    ref = brute.direct_sum(t.xyz(), s.xyz(), s.q, "poly")
    assert core.rel_l2(phi, ref) < 1e-13


@pytest.mark.parametrize("scheme", ["bltc", "cp_bltc"])
def test_treecode_tiny_theta_is_the_direct_sum(scheme):
    p = inputs.particles(2000, seed=67)
    run = core.Run(p, p, theta=1e-9, degree=2, leaf=100, scheme=scheme)
    phi = run.run_all()
    L = run.lists()
    leaves = int(np.sum(run.tree(0)["nchild"] == 0))
    assert all(len(L[k][0]) == 0 for k in ("PC", "CP", "CC")) and len(L["PP"][0]) == leaves ** 2
    assert core.rel_l2(phi, core.direct_sum(p, p)) < 1e-14


def test_treecodes_differ_from_the_dual_tree_at_the_approximation_level():
    # Sec. 4.2: at one (theta, n) the three methods are approximations of the
    # same sum, of comparable error; the error falls with n for the treecodes too
    p = inputs.particles(20000, seed=69)
    sel = inputs.error_sample(20000, 69, fraction=0.05)
    ref = core.direct_sum(p, p, sel=sel)
    errs = {}
    for scheme in ("bldtt", "bltc", "cp_bltc"):
        e = [core.rel_l2(core.bldtt(p, p, theta=0.7, degree=n, leaf=100, scheme=scheme)[sel], ref) for n in (2, 4, 6)]
        assert e[0] > e[1] > e[2], (scheme, e)
        errs[scheme] = e
    for n_i in range(3):
        vals = [errs[k][n_i] for k in errs]
        assert max(vals) < 10 * min(vals), errs


def test_lists_tiny_theta_gives_leaf_leaf_pp_only():
    p = inputs.particles(2000, seed=9)
    run = core.Run(p, p, theta=1e-9, degree=2, leaf=100)
    run.traverse()
    L = run.lists()
    tree = run.tree(0)
    leaves = np.flatnonzero(tree["nchild"] == 0)
    assert all(len(L[k][0]) == 0 for k in ("PC", "CP", "CC"))
    assert len(L["PP"][0]) == len(leaves) ** 2


def test_lists_large_np_no_approximations():
    p = inputs.particles(700, seed=10)
    run = core.Run(p, p, theta=0.9, degree=9, leaf=10)      # (n+1)^3 = 1000 >= N
    run.traverse()
    L = run.lists()
    assert all(len(L[k][0]) == 0 for k in ("PC", "CP", "CC"))


def test_lists_two_far_clusters_hand_case():
    # two tight blobs of 400 points, 10 apart: each a child of the root; they separate at theta 0.5
    rng = np.random.default_rng(12)
    a = rng.uniform(-0.5, 0.5, (400, 3))
    b = a + np.array([10.0, 0.0, 0.0])
    xyz = np.vstack([a, b])
    p = inputs.ParticleSet(*[xyz[:, d].copy() for d in range(3)], q=np.ones(800))
    run = core.Run(p, p, theta=0.5, degree=2, leaf=400)        # n_p = 27
    run.traverse()
    L = run.lists()
    tree = run.tree(0)
    assert tree["nchild"][0] == 2
    c1, c2 = tree["child"][0][:2]
    cc = set(zip(*L["CC"]))
    assert cc == {(c1, c2), (c2, c1)}
    pp = set(zip(*L["PP"]))
    assert pp == {(c1, c1), (c2, c2)}


# --------------------------------------------------------------------------
# Upward pass (Sec. 2.5, Appendix B), downward pass (Sec. 2.7, Appendix C)
# --------------------------------------------------------------------------

def test_upward_leaf_preserves_moments():
    # sum_k qhat_k p(s_k) = sum_j q_j p(y_j) for tensor monomials of degree <= n per coordinate
    n = 4
    p = inputs.particles(3000, "gaussian", seed=13)
    run = core.Run(p, p, theta=0.7, degree=n, leaf=200)
    run.upward()
    qh = run.qhat()
    tree = run.tree(1)
    for c in range(0, tree["lo"].shape[0], 7):
        S = brute.grid3(n, tree["lo"][c], tree["hi"][c])
        idx = tree["perm"][tree["begin"][c]:tree["begin"][c] + tree["count"][c]]
        Y = p.xyz()[idx]
        for a, b, d in ((0, 0, 0), (1, 0, 0), (0, 2, 1), (4, 4, 4), (3, 1, 2)):
            lhs = qh[c] @ (S[:, 0] ** a * S[:, 1] ** b * S[:, 2] ** d)
            rhs = p.q[idx] @ (Y[:, 0] ** a * Y[:, 1] ** b * Y[:, 2] ** d)
            assert abs(lhs - rhs) <= 1e-12 * max(1.0, np.abs(p.q[idx]).sum())


@pytest.mark.parametrize("dist,n", [("uniform", 3), ("gaussian", 6), ("sphere", 8)])
def test_upward_recursive_equals_direct_form(dist, n):
    p = inputs.particles(6000, dist, seed=14)
    run = core.Run(p, p, theta=0.7, degree=n, leaf=150)
    run.upward()
    rec, direct = run.qhat(), run.qhat_direct()
    scale = np.abs(direct).max()
    assert np.abs(rec - direct).max() <= 1e-13 * scale * 10


def _far_targets(m, n, seed):
    # a target blob far from the sources: the target root itself takes CP/CC entries
    t, s = inputs.unequal_sets(m, "sphere", n, "uniform", seed=seed)
    t = inputs.ParticleSet(0.5 * t.x + 4.0, 0.5 * t.y, 0.5 * t.z)
    return t, s


@pytest.mark.parametrize("dist,n", [("uniform", 3), ("gaussian", 5), ("far", 4)])
def test_downward_recursive_equals_direct_chain_form(dist, n):
    if dist == "far":
        t, s = _far_targets(5000, 6000, 15)
    else:
        t, s = inputs.unequal_sets(5000, dist, 6000, "uniform", seed=15)
    run = core.Run(t, s, theta=0.6, degree=n, leaf=60)
    run.run_all()
    rec = run.potentials()
    direct = run.downward_direct()
    assert core.rel_l2(rec, direct) < 1e-13


# --------------------------------------------------------------------------
# Whole pipeline
# --------------------------------------------------------------------------

@pytest.mark.parametrize("theta", [0.5, 0.7, 0.95])
@pytest.mark.parametrize("n", [2, 3])
def test_polynomial_kernel_is_reproduced_exactly(theta, n):
    # G = (1 + x.y)^2 has degree 2 per coordinate: every approximation type is exact for n >= 2
    t, s = inputs.unequal_sets(2500, "uniform", 3000, "gaussian", seed=16)
    run = core.Run(t, s, kernel="poly", theta=theta, degree=n, leaf=40)
    phi = run.run_all()
    counts = {k: len(v[0]) for k, v in run.lists().items()}
    assert counts["CC"] + counts["PC"] + counts["CP"] > 0
    ref = brute.direct_sum(t.xyz(), s.xyz(), s.q, "poly")
    assert core.rel_l2(phi, ref) < 1e-13


def test_polynomial_kernel_degree_one_is_not_exact():
    # sanity: the same check fails when the interpolant cannot hold the kernel
    t, s = inputs.unequal_sets(2500, "uniform", 3000, "gaussian", seed=16)
    run = core.Run(t, s, kernel="poly", theta=0.7, degree=1, leaf=40)
    phi = run.run_all()
    ref = brute.direct_sum(t.xyz(), s.xyz(), s.q, "poly")
    assert core.rel_l2(phi, ref) > 1e-8


@pytest.mark.parametrize("kernel", ["coulomb", "yukawa", "oscillatory", "regcoulomb"])
@pytest.mark.parametrize("case", ["same", "unequal"])
def test_explicit_matrix_brute_force(kernel, case):
    # sum over list entries of explicit approximated-kernel matrices (no up/down passes)
    if case == "same":
        t = s = inputs.particles(1200, "gaussian", seed=17)
    else:
        t, s = inputs.unequal_sets(900, "sphere", 1300, "gaussian", seed=18)
    n = 2
    run = core.Run(t, s, kernel=kernel, theta=0.9, degree=n, leaf=20)
    phi = run.run_all()
    counts = {k: len(v[0]) for k, v in run.lists().items()}
    assert min(counts.values()) > 0, counts            # all four types exercised
    ref = brute.explicit_bldtt(t.xyz(), s.xyz(), s.q, run.tree(0), run.tree(1), run.lists(), n, kernel,
                               core.DEFAULT_PARAM[kernel])
    assert core.rel_l2(phi, ref) < 1e-13


def test_leaf_at_least_n_gives_direct_sum():
    p = inputs.particles(3000, seed=19)
    phi = core.bldtt(p, p, theta=0.7, degree=4, leaf=3000)
    ref = core.direct_sum(p, p)
    assert core.rel_l2(phi, ref) < 1e-14


def test_error_falls_as_degree_rises():
    # Sec. 4.3: at fixed theta the error decreases as n increases
    p = inputs.particles(20000, seed=20)
    sel = inputs.error_sample(20000, 20, fraction=0.05)
    ref = core.direct_sum(p, p, sel=sel)
    errs = []
    for n in (1, 2, 4, 6, 8):
        phi = core.bldtt(p, p, theta=0.7, degree=n, leaf=100)
        errs.append(core.rel_l2(phi[sel], ref))
    assert all(b < a for a, b in zip(errs, errs[1:])), errs
    assert errs[-1] < 1e-6


@pytest.mark.slow
def test_error_magnitude_matches_paper_table():
    # Table pc_cc_scaling: 1.58e-8 at N = 1E5, theta 0.7, n 8, leaf 2000; band of x5
    g = json.load(open(os.path.join(GOLDEN, "paper_table_pc_cc_scaling.json")))
    N = 100_000
    p = inputs.particles(N, seed=21)
    phi = core.bldtt(p, p, theta=g["theta"], degree=g["degree"], leaf=g["leaf"])
    sel = inputs.error_sample(N, 21, fraction=0.01)
    err = core.rel_l2(phi[sel], core.direct_sum(p, p, sel=sel))
    paper = g["bldtt_error"][str(N)]
    assert paper / 5 < err < paper * 5, err


def test_eval_targets_equals_full_run():
    t, s = inputs.unequal_sets(4000, "uniform", 5000, "gaussian", seed=22)
    run = core.Run(t, s, theta=0.7, degree=4, leaf=50)
    phi = run.run_all()
    sel = np.array([0, 7, 3999, 1234, 2500])
    got = run.eval_targets(sel)
    assert core.rel_l2(got, phi[sel]) < 1e-13


# --------------------------------------------------------------------------
# Per-pair degrees: lists whose approximated entries carry their own degree
# --------------------------------------------------------------------------

def test_per_entry_degree_evaluator_equals_standard_run_at_one_degree():
    # every entry at the run's degree: the direct chain form must equal the recursive run
    t, s = inputs.unequal_sets(3000, "sphere", 4000, "gaussian", seed=23)
    run = core.Run(t, s, theta=0.8, degree=4, leaf=40)
    phi = run.run_all()
    L = {k: (tc, sc, np.full(tc.shape[0], 4, np.int32)) for k, (tc, sc) in run.lists().items()}
    got = run.eval_degrees(L)
    assert core.rel_l2(got, phi) < 1e-13


def test_per_entry_degree_evaluator_vs_explicit_matrices():
    # mixed degrees per entry (2..7): the oracle's evaluator against the explicit approximated matrices
    t, s = inputs.unequal_sets(900, "sphere", 1300, "gaussian", seed=24)
    run = core.Run(t, s, theta=0.9, degree=2, leaf=20)
    run.traverse()
    rng = np.random.default_rng(24)
    L = {k: (tc, sc, rng.integers(2, 8, size=tc.shape[0]).astype(np.int32)) for k, (tc, sc) in run.lists().items()}
    assert min(len(v[0]) for v in L.values()) > 0
    got = run.eval_degrees(L)
    ref = brute.explicit_bldtt(t.xyz(), s.xyz(), s.q, run.tree(0), run.tree(1), L, 2)
    assert core.rel_l2(got, ref) < 1e-13


# --------------------------------------------------------------------------
# The FP64 reference of the degree model: backpropagation against central
# finite differences, and the network's closed forms.
# --------------------------------------------------------------------------

def _random_model(seed, scale=0.3):
    from oracle import mlp
    rng = np.random.default_rng(seed)
    m = rng.normal(0, scale, mlp.N_MODEL)
    m[mlp.N_PARAMS:mlp.N_PARAMS + 4] = rng.normal(0, 1, 4)        # mean
    m[mlp.N_PARAMS + 4:mlp.N_PARAMS + 8] = rng.uniform(0.5, 2, 4)  # scale
    return m


def test_mlp_reference_gradient_matches_finite_differences():
    from oracle import mlp
    rng = np.random.default_rng(30)
    model = _random_model(30)
    f = rng.normal(0, 1, (17, 4))
    t = rng.normal(-6, 2, (17, 11))
    t[3, 5] = np.nan                      # missing targets are ignored
    g = mlp.grad(model, f, t)
    h = 1e-6
    for q in rng.choice(mlp.N_PARAMS, size=60, replace=False):
        mp, mm = model.copy(), model.copy()
        mp[q] += h
        mm[q] -= h
        fd = (mlp.loss(mp, f, t) - mlp.loss(mm, f, t)) / (2 * h)
        assert abs(fd - g[q]) <= 1e-7 + 1e-6 * abs(fd), (q, fd, g[q])


def test_mlp_reference_closed_forms():
    from oracle import mlp
    model = np.zeros(mlp.N_MODEL)
    model[mlp.N_PARAMS + 4:mlp.N_PARAMS + 8] = 1.0
    p = mlp.unpack(model)
    p["b3"][:] = np.arange(11)           # views into model
    y, _ = mlp.forward(model, np.ones((3, 4)))
    assert np.array_equal(y, np.tile(np.arange(11.0), (3, 1)))
    # a single path: y_0 = W3[0,0] tanh(W2[0,0] tanh(W1[0,0] x0))
    p["W1"][0, 0], p["W2"][0, 0], p["W3"][0, 0] = 0.5, -1.5, 2.0
    y, _ = mlp.forward(model, np.array([[0.8, 0.0, 0.0, 0.0]]))
    assert y[0, 0] == pytest.approx(2.0 * np.tanh(-1.5 * np.tanh(0.5 * 0.8)), rel=1e-15)
