"""Seeded synthetic particle sets for the BLDTT workloads.

This module is the only code shared by the HIP path, the CPU oracle, the
tests and the benchmark.  It draws random numbers and nothing else: no
interpolation, no kernel evaluation, no tree logic.

The distributions follow the paper's experiments (Sec. 4): particles uniform
in [-1,1]^3 with charges uniform in [-1,1] (problem-size scaling, Sec. 4.1),
a Gaussian cloud (Sec. 4.3, read as N(0, 0.25^2) per coordinate), and points
uniform on the unit sphere (non-cubic domains, Sec. 4.4).

Every array is float64, C-contiguous, split into structure-of-arrays
(x, y, z, q).  Generators are numpy PCG64 streams; positions are drawn as an
(n, 3) block first and the charges after them.
"""
from __future__ import annotations

import dataclasses

import numpy as np

BASE_SEED = 20126925


@dataclasses.dataclass
class ParticleSet:
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    q: np.ndarray | None = None

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    def xyz(self) -> np.ndarray:
        return np.stack([self.x, self.y, self.z], axis=1)


def _split(pos: np.ndarray, q: np.ndarray | None) -> ParticleSet:
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    return ParticleSet(np.ascontiguousarray(pos[:, 0]),
                       np.ascontiguousarray(pos[:, 1]),
                       np.ascontiguousarray(pos[:, 2]),
                       None if q is None else np.ascontiguousarray(q, dtype=np.float64))


def _positions(rng: np.random.Generator, n: int, dist: str) -> np.ndarray:
    if dist == "uniform":
        return rng.uniform(-1.0, 1.0, size=(n, 3))
    if dist == "gaussian":
        return rng.normal(0.0, 0.25, size=(n, 3))
    if dist == "sphere":
        v = rng.normal(0.0, 1.0, size=(n, 3))
        return v / np.linalg.norm(v, axis=1, keepdims=True)
    if dist == "slab":          # 1 x 10 x 10 box
        return rng.uniform(0.0, 1.0, size=(n, 3)) * np.array([1.0, 10.0, 10.0])
    if dist == "rod":           # 1 x 1 x 10 box
        return rng.uniform(0.0, 1.0, size=(n, 3)) * np.array([1.0, 1.0, 10.0])
    if dist == "plummer":
        # radial density 3/(4 pi) (1 + r^2)^(-5/2) (Sec. 4.3): the mass inside r is
        # r^3 / (1 + r^2)^(3/2), inverted for r; isotropic directions; points with
        # a coordinate beyond +-100 are drawn again
        out = np.empty((0, 3))
        while out.shape[0] < n:
            m = n - out.shape[0]
            u = rng.uniform(0.0, 1.0, size=m)
            with np.errstate(divide="ignore"):
                r = 1.0 / np.sqrt(u ** (-2.0 / 3.0) - 1.0)
            v = rng.normal(0.0, 1.0, size=(m, 3))
            v *= (r / np.linalg.norm(v, axis=1))[:, None]
            out = np.concatenate([out, v[np.all(np.abs(v) <= 100.0, axis=1)]])
        return out
    raise ValueError(f"unknown distribution {dist!r}")


def particles(n: int, dist: str = "uniform", seed: int = BASE_SEED, charges: bool = True) -> ParticleSet:
    """n particles of one distribution; charges U[-1,1] drawn after positions
    (Plummer particles carry 1/n each, as in Sec. 4.3)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    pos = _positions(rng, n, dist)
    if not charges:
        q = None
    elif dist == "plummer":
        q = np.full(n, 1.0 / n)
    else:
        q = rng.uniform(-1.0, 1.0, size=n)
    return _split(pos, q)


# Error target of the per-pair degree choice (one value for every workload): the largest tau in a
# sweep whose global relative l2 error stays at or below 1e-6 at both 1E7 and 1E8 (1e-6 gives
# 1.01e-6 at 1E8, theta 0.87).
TAU = 7e-7

# Named workloads.  'id' offsets the base seed so every workload has its own stream.
WORKLOADS = {
    # targets = sources, uniform cube, Coulomb, theta 0.7, n 6, leaf 500
    "cube1e4": dict(id=1, M=10_000, dist="uniform", kernel="coulomb", theta=0.7, degree=6, leaf=500),
    # targets = sources, uniform cube, Coulomb, theta 0.8, n 8, leaf 2000
    "cube1e6": dict(id=2, M=1_000_000, dist="uniform", kernel="coulomb", theta=0.8, degree=8, leaf=2000, tau=TAU),
    # unequal: Gaussian sources, sphere-surface targets, Yukawa kappa 0.5
    "sphere2e6_gauss1e7": dict(id=3, M=2_000_000, N=10_000_000, tdist="sphere", sdist="gaussian",
                               kernel="yukawa", theta=0.7, degree=8, leaf=2000),
    # targets = sources, uniform cube 1E7, Coulomb (the throughput workload).  theta and degree are
    # the fastest plain-FP64 pair with relative l2 error <= 1e-6 in a theta x degree sweep at leaf 2000.
    # tuned_theta: the fastest theta of the FP32-evaluation + per-pair-degree form with error <= 1e-6
    # in a theta x tau sweep.
    "cube1e7": dict(id=0, M=10_000_000, dist="uniform", kernel="coulomb", theta=0.8, degree=7, leaf=2000,
                    tuned_theta=0.87, tau=TAU, tuned_fallback=8),
    # 1E8: the learned-degree form at the workload's theta 0.8 and at the faster 0.87
    "cube1e8": dict(id=5, M=100_000_000, dist="uniform", kernel="coulomb", theta=0.8, degree=8, leaf=2000,
                    tuned_theta=0.87, tau=TAU, tuned_fallback=8),
    # 256 independent targets = sources problems, sizes log-uniform in [1E3, 1E5], distribution per
    # problem from {uniform cube, Gaussian, sphere surface}; Coulomb, theta 0.7, n 6, leaf 500
    "batch256": dict(id=4, count=256, lo_exp=3.0, hi_exp=5.0, kernel="coulomb", theta=0.7, degree=6, leaf=500),
}


def workload_seed(name: str) -> int:
    return BASE_SEED + WORKLOADS[name]["id"]


def same_set(n: int, dist: str, seed: int) -> ParticleSet:
    """Targets = sources: one set with charges."""
    return particles(n, dist, seed, charges=True)


def unequal_sets(m: int, tdist: str, n: int, sdist: str, seed: int) -> tuple[ParticleSet, ParticleSet]:
    """Distinct target (no charges) and source (with charges) sets from one seed."""
    ss = np.random.SeedSequence(seed)
    ts, sr = ss.spawn(2)
    rt = np.random.Generator(np.random.PCG64(ts))
    rs = np.random.Generator(np.random.PCG64(sr))
    tgt = _split(_positions(rt, m, tdist), None)
    spos = _positions(rs, n, sdist)
    src = _split(spos, rs.uniform(-1.0, 1.0, size=n))
    return tgt, src


def batch_problems(count: int = 256, seed: int = BASE_SEED + 4, lo_exp: float = 3.0, hi_exp: float = 5.0,
                   dists=("uniform", "gaussian", "sphere")) -> list[tuple[str, ParticleSet]]:
    """Many independent targets=sources problems with log-uniform sizes.

    Sizes are round(10**U(lo_exp, hi_exp)); each problem's distribution is drawn
    uniformly from `dists`; per-problem streams come from SeedSequence.spawn.
    """
    ss = np.random.SeedSequence(seed)
    top = np.random.Generator(np.random.PCG64(ss))
    sizes = np.rint(10.0 ** top.uniform(lo_exp, hi_exp, size=count)).astype(np.int64)
    kinds = top.integers(0, len(dists), size=count)
    out = []
    for child, n, k in zip(ss.spawn(count), sizes, kinds):
        rng = np.random.Generator(np.random.PCG64(child))
        pos = _positions(rng, int(n), dists[int(k)])
        q = rng.uniform(-1.0, 1.0, size=int(n))
        out.append((dists[int(k)], _split(pos, q)))
    return out


def error_sample(m: int, seed: int, fraction: float = 1e-3, minimum: int = 1) -> np.ndarray:
    """Indices of the random target subset used for the error (sampled without replacement)."""
    k = max(minimum, int(m * fraction))
    k = min(k, m)
    rng = np.random.Generator(np.random.PCG64(seed + 1000))
    return np.sort(rng.choice(m, size=k, replace=False)).astype(np.int64)
