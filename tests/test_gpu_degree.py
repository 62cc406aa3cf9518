"""Per-pair interpolation degree on the GPU: the degree machinery against the
oracle's per-entry-degree evaluator, the MLP kernels against the FP64
reference, the measured pair errors against explicit matrices, and training."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import brute, core, mlp  # noqa: E402
from paper_2012_06925_amd import inputs  # noqa: E402

LEARNED = 2
FP32 = 1
FP32_MIXED = 4e-7      # FP32 evaluation against the FP64 oracle, degrees 2..12 mixed (measured 9.9e-8, 1.1e-7)


def _api():
    from paper_2012_06925_amd import api
    return api


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _plan(t, s, same, **kw):
    api = _api()
    src = [dev(a) for a in (s.x, s.y, s.z, s.q)]
    tgt = None if same else [dev(a) for a in (t.x, t.y, t.z)]
    return api.Plan(tgt, src, **kw)


def _lists_with_degrees(plan):
    L, D = plan.lists(), plan.list_degrees()
    return {k: (L[k][0], L[k][1], D[k]) for k in L}


@pytest.mark.parametrize("case", ["same", "unequal"])
def test_mixed_degrees_match_oracle(case):
    # every separated pair at degree 2 + (7 tc + 13 sc) mod 11: all degrees 2..12 mixed
    if case == "same":
        t = s = inputs.particles(20_000, "gaussian", seed=70)
    else:
        t, s = inputs.unequal_sets(15_000, "sphere", 20_000, "uniform", seed=71)
    plan = _plan(t, s, case == "same", theta=0.8, degree=6, leaf=60, flags=LEARNED)
    plan.set_degree_test_rule()
    phi = plan.compute().cpu().numpy()
    L = _lists_with_degrees(plan)
    tree_t, tree_s = plan.tree(0), plan.tree(1)
    for name in ("PC", "CP", "CC"):
        tc, sc, dg = L[name]
        assert np.array_equal(dg, 2 + (7 * tc + 13 * sc) % 11), name
        npx = (dg + 1) ** 3
        ct, cs = tree_t["count"][tc], tree_s["count"][sc]
        if name == "CC":
            assert np.all((ct > npx) & (cs > npx))
    st = plan.stats()
    assert bin(st["degree_mask"]).count("1") >= 8, st
    run = core.Run(t, s, theta=0.8, degree=6, leaf=60, aliased=case == "same")
    ref = run.eval_degrees(L)
    err = core.rel_l2(phi, ref)
    print(f"\n  mixed degrees {case}: mask={st['degree_mask']:#x} down={st['down_degree']} gpu-vs-oracle={err:.2e}")
    assert err < 1e-12 and core.max_rel(phi, ref) < 1e-12
    # the next compute forms the charges of the last compute's degrees before
    # the traversal (the largest from the particles, the rest by restriction)
    phi2 = plan.compute().cpu().numpy()
    assert core.rel_l2(phi2, ref) < 1e-12 and core.max_rel(phi2, ref) < 1e-12


@pytest.mark.parametrize("case", ["same", "unequal"])
def test_mixed_degrees_fp32_evaluation(case):
    # the same degree rule with FP32 evaluation: targets = sources runs the
    # symmetric passes on the matrix cores for PP and for the CC pairs whose
    # two directions share a degree (proxy tiles of 27 .. 2197 points), the
    # rest one-sided; within the FP32 bound of the FP64 per-entry-degree oracle
    if case == "same":
        t = s = inputs.particles(20_000, "gaussian", seed=70)
    else:
        t, s = inputs.unequal_sets(15_000, "sphere", 20_000, "uniform", seed=71)
    plan = _plan(t, s, case == "same", theta=0.8, degree=6, leaf=60, flags=LEARNED | FP32)
    plan.set_degree_test_rule()
    phi = plan.compute().cpu().numpy()
    L = _lists_with_degrees(plan)
    st = plan.stats()
    if case == "same":
        assert st["pass_interactions"][2] > 0 and st["pass_interactions"][3] > 0, st["pass_interactions"]
    run = core.Run(t, s, theta=0.8, degree=6, leaf=60, aliased=case == "same")
    err = core.rel_l2(phi, run.eval_degrees(L))
    print(f"\n  mixed degrees FP32 {case}: gpu-vs-oracle={err:.2e}")
    assert err < FP32_MIXED


@pytest.mark.parametrize("case", ["same", "unequal"])
def test_model_choice_matches_oracle(case):
    # the committed model chooses the degrees (its inference on the GPU, ahead
    # of the near-field pass for a problem this small); the potentials equal
    # the oracle's per-entry-degree evaluation of the chosen lists
    from paper_2012_06925_amd.train_degree_model import load_model
    if case == "same":
        t = s = inputs.particles(40_000, "uniform", seed=80)
    else:
        t, s = inputs.unequal_sets(15_000, "sphere", 40_000, "gaussian", seed=81)
    plan = _plan(t, s, case == "same", theta=0.8, degree=6, leaf=200, flags=LEARNED)
    plan.set_degree_model(load_model(), fallback=6, tau=1e-6)
    phi = plan.compute().cpu().numpy()
    st = plan.stats()
    assert st["sep_pairs"] > 0 and sum(st["pairs_per_degree"].values()) + st["sep_direct"] == st["sep_pairs"], st
    L = _lists_with_degrees(plan)
    run = core.Run(t, s, theta=0.8, degree=6, leaf=200, aliased=case == "same")
    ref = run.eval_degrees(L)
    err = core.rel_l2(phi, ref)
    print(f"\n  model choice {case}: degrees {st['pairs_per_degree']} direct {st['sep_direct']} gpu-vs-oracle={err:.2e}")
    assert err < 1e-12 and core.max_rel(phi, ref) < 1e-12
    # a second compute chooses the same degrees and gives the same potentials
    # (to rounding: it restricts charges the first formed from the particles);
    # from then on every compute gives the same bits
    phi2 = plan.compute().cpu().numpy()
    assert core.rel_l2(phi2, phi) < 1e-13
    phi3 = plan.compute().cpu().numpy()
    assert np.array_equal(phi2, phi3)


def test_tuned_form_recompute_is_bit_identical():
    # the timed tuned form (FP32 evaluation, learned degree, symmetric passes
    # with their folds): computes after the first give the same bits
    from paper_2012_06925_amd.train_degree_model import load_model
    p = inputs.particles(80_000, "uniform", seed=inputs.BASE_SEED + 342)
    plan = _plan(p, p, True, theta=0.87, degree=8, leaf=400, flags=LEARNED | FP32)
    plan.set_degree_model(load_model(), fallback=8, tau=7e-7)
    phis = [plan.compute().cpu().numpy() for _ in range(4)]
    st = plan.stats()
    plan.close()
    assert st["pass_interactions"][2] > 0
    for later in phis[2:]:
        assert np.array_equal(phis[1], later)
    ref = core.bldtt(p, p, theta=0.87, degree=8, leaf=400)
    assert core.rel_l2(phis[1], ref) < 1e-5


def test_fallback_policy_equals_plain_method():
    p = inputs.particles(30_000, "uniform", seed=72)
    plain = _plan(p, p, True, theta=0.7, degree=5, leaf=150)
    varied = _plan(p, p, True, theta=0.7, degree=5, leaf=150, flags=LEARNED)
    varied.set_degree_model(None, fallback=5, tau=1e-6)
    a = plain.compute().cpu().numpy()
    b = varied.compute().cpu().numpy()
    assert core.rel_l2(b, a) < 1e-13
    for k in ("PP", "PC", "CP", "CC"):
        assert sorted(zip(*plain.lists()[k])) == sorted(zip(*varied.lists()[k]))


def test_mlp_forward_matches_fp64_reference():
    api = _api()
    rng = np.random.default_rng(73)
    model = rng.normal(0, 0.3, api.mlp_model_size()).astype(np.float32)
    model[mlp.N_PARAMS:mlp.N_PARAMS + 4] = rng.normal(0, 1, 4)
    model[mlp.N_PARAMS + 4:mlp.N_PARAMS + 8] = rng.uniform(0.5, 2, 4)
    f = rng.normal(0, 2, (5000, 4)).astype(np.float32)
    got = api.mlp_forward(dev(model), dev(f)).cpu().numpy()
    ref, _ = mlp.forward(model.astype(np.float64), f.astype(np.float64))
    assert np.abs(got - ref).max() <= 2e-5 * max(1.0, np.abs(ref).max())


def test_mlp_gradient_matches_fp64_reference():
    # the project's backward kernels against backpropagation in FP64 (itself pinned by finite differences)
    api = _api()
    rng = np.random.default_rng(74)
    model = rng.normal(0, 0.3, api.mlp_model_size()).astype(np.float32)
    model[mlp.N_PARAMS:mlp.N_PARAMS + 4] = rng.normal(0, 1, 4)
    model[mlp.N_PARAMS + 4:mlp.N_PARAMS + 8] = rng.uniform(0.5, 2, 4)
    f = rng.normal(0, 1.5, (700, 4)).astype(np.float32)
    t = rng.normal(-6, 2, (700, 11)).astype(np.float32)
    t[rng.random(t.shape) < 0.05] = np.nan
    loss, g = api.mlp_loss_grad(dev(model), dev(f), dev(t))
    g = g.cpu().numpy()
    m64 = model.astype(np.float64)
    ref_loss = mlp.loss(m64, f.astype(np.float64), t.astype(np.float64))
    ref = mlp.grad(m64, f.astype(np.float64), t.astype(np.float64))
    assert loss == pytest.approx(ref_loss, rel=1e-5)
    assert np.linalg.norm(g - ref) <= 1e-4 * np.linalg.norm(ref)


def test_pair_errors_match_explicit_matrices():
    # the GPU-measured error of a pair's cluster-cluster approximation at degree d
    # against explicit approximated matrices (NumPy, product-form Lagrange)
    t = s = inputs.particles(4000, "uniform", seed=75)
    plan = _plan(t, s, True, theta=0.8, degree=4, leaf=64)
    feats, errs, pairs = plan.pair_errors(with_pairs=True)
    tree = plan.tree(0)
    assert feats.shape[0] > 50 and errs.shape == (feats.shape[0], 11)
    # every listed pair is separated by the MAC
    c = tree["center"]
    R = np.linalg.norm(c[pairs[:, 0]] - c[pairs[:, 1]], axis=1)
    assert np.all((tree["radius"][pairs[:, 0]] + tree["radius"][pairs[:, 1]]) / R < 0.8)
    np.testing.assert_allclose(feats[:, 2], np.log(tree["count"][pairs[:, 0]]), rtol=1e-6)
    rng = np.random.default_rng(75)
    xyz = t.xyz()
    for k in rng.choice(feats.shape[0], size=10, replace=False):
        tc, sc = pairs[k]
        ti = tree["perm"][tree["begin"][tc]:tree["begin"][tc] + tree["count"][tc]]
        exact = brute.explicit_bldtt(xyz, xyz, t.q, tree, tree, {"PP": ([tc], [sc])}, 2)[ti]
        for d in (2, 5, 9):
            approx = brute.explicit_bldtt(xyz, xyz, t.q, tree, tree, {"CC": ([tc], [sc], [d])}, d)[ti]
            e = np.linalg.norm(approx - exact) / np.linalg.norm(exact)
            want = np.log10(max(e, 1e-14))
            tol = 1e-3 if e > 1e-12 else 0.5
            assert abs(errs[k, d - 2] - want) < tol, (tc, sc, d, e, errs[k, d - 2])


def test_training_on_measured_errors():
    api = _api()
    feats, errs = [], []
    for dist, seed in (("uniform", 76), ("gaussian", 77)):
        p = inputs.particles(100_000, dist, seed=seed)
        plan = _plan(p, p, True, theta=0.9, degree=8, leaf=500)
        f, e = plan.pair_errors()
        feats.append(f)
        errs.append(e)
    f = np.concatenate(feats)
    e = np.concatenate(errs)
    model, hist = api.mlp_train(f, e, epochs=150, batch=512, lr=2e-3, seed=1)
    print(f"\n  {f.shape[0]} pairs; loss {hist[0]:.3f} -> {hist[-1]:.4f}")
    assert np.all(np.isfinite(hist)) and hist[-1] < 0.1 * hist[0]
    pred = api.mlp_forward(dev(model), dev(f)).cpu().numpy()
    ok = ~np.isnan(e)
    rmse = float(np.sqrt(np.mean((pred[ok] - e[ok]) ** 2)))
    # baseline without the pair features: the mean error of each degree
    base = np.where(ok, np.nanmean(e, axis=0, keepdims=True), np.nan)
    rmse0 = float(np.sqrt(np.mean((base[ok] - e[ok]) ** 2)))
    print(f"  training rmse (log10 units) {rmse:.3f}; per-degree mean {rmse0:.3f}")
    assert rmse < 0.6 and rmse < 0.5 * rmse0


@pytest.mark.parametrize("dist", ["uniform", "gaussian"])
def test_learned_degree_gain_over_fallback(dist):
    # The committed model (trained on seeds >= 20127000) on an unseen problem:
    # at the same theta it must meet the 1e-6 target with fewer kernel
    # evaluations in all (PP included) than every separated pair at the
    # fallback degree 8.  (At degree 8 Algorithm 2 sends most separated pairs
    # of 500-particle leaves to PP; lower learned degrees make them PC/CP/CC.)
    from paper_2012_06925_amd import _lib
    from paper_2012_06925_amd.train_degree_model import load_model
    api = _api()
    p = inputs.particles(300_000, dist, seed=79)
    src = [dev(a) for a in (p.x, p.y, p.z, p.q)]
    sel = inputs.error_sample(p.n, 79, fraction=5e-3)
    ref = api.direct_sum(src[:3], src, sel=dev(sel)).cpu().numpy()

    def run(flags, model=None):
        plan = api.Plan(None, src, theta=0.8, degree=8, leaf=500, flags=flags)
        if model is not None:
            plan.set_degree_model(model, fallback=8, tau=1e-6)
        phi = plan.compute().cpu().numpy()
        st = plan.stats()
        plan.close()
        err = float(np.sqrt(np.sum((phi[sel] - ref) ** 2) / np.sum(ref ** 2)))
        approx = sum(st["interactions"][k] for k in ("PC", "CP", "CC"))
        return err, approx, sum(st["interactions"].values()), st

    e_fixed, a_fixed, t_fixed, _ = run(0)
    e_learn, a_learn, t_learn, st = run(_lib.LEARNED_DEGREE, load_model())
    print(f"\n  fixed n=8: err {e_fixed:.2e}, approx evals {a_fixed:.3e}, all {t_fixed:.3e}"
          f"\n  learned:   err {e_learn:.2e}, approx evals {a_learn:.3e}, all {t_learn:.3e}, "
          f"degrees {st['pairs_per_degree']}, direct {st['sep_direct']}, fallback {st['sep_fallback']}")
    assert e_learn <= 1e-6 and e_learn <= max(e_fixed, 1e-6)
    assert t_learn < 0.9 * t_fixed              # measured: 0.68 (uniform), 0.82 (Gaussian)
    assert st["sep_fallback"] < 0.01 * st["sep_pairs"]
