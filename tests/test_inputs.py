"""The seeded input generator against the distributions it claims to draw
(no method arithmetic here: these pin the inputs every other test uses)."""
import numpy as np

from paper_2012_06925_amd import inputs


def test_plummer_radial_law_cutoff_and_charges():
    # Sec. 4.3: radial density 3/(4 pi) (1 + r^2)^(-5/2), so the fraction of
    # particles inside r is r^3 / (1 + r^2)^(3/2); every coordinate within
    # +-100; charges 1/N
    n = 200_000
    p = inputs.particles(n, "plummer", seed=5)
    xyz = p.xyz()
    assert np.all(np.abs(xyz) <= 100.0)
    assert np.allclose(p.q, 1.0 / n) and abs(p.q.sum() - 1.0) < 1e-9
    r = np.sort(np.linalg.norm(xyz, axis=1))
    grid = np.array([0.1, 0.3, 0.5, 0.77, 1.0, 1.5, 2.0, 3.0, 5.0, 10.0, 30.0])
    emp = np.searchsorted(r, grid) / n
    law = grid ** 3 / (1.0 + grid ** 2) ** 1.5
    assert np.max(np.abs(emp - law)) < 5e-3, np.max(np.abs(emp - law))
    # isotropy: the mean position is near zero, each axis carries a third of r^2
    assert np.all(np.abs(xyz.mean(axis=0)) < 0.05)
    share = (xyz ** 2).sum(axis=0) / (xyz ** 2).sum()
    assert np.all(np.abs(share - 1.0 / 3.0) < 0.05)


def test_uniform_and_gaussian_moments_and_seeding():
    a = inputs.particles(100_000, "uniform", seed=7)
    b = inputs.particles(100_000, "uniform", seed=7)
    assert np.array_equal(a.x, b.x) and np.array_equal(a.q, b.q)
    assert a.x.min() >= -1.0 and a.x.max() < 1.0
    assert abs(a.x.var() - 1.0 / 3.0) < 0.01 and abs(a.q.mean()) < 0.01
    g = inputs.particles(100_000, "gaussian", seed=8)
    assert abs(g.y.std() - 0.25) < 0.005
