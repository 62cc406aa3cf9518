"""Independent NumPy brute-force forms for tiny inputs (test infrastructure only).

These deliberately avoid the barycentric machinery of the C oracle so they
can pin it:
  * Chebyshev points as cos(pi k / n) and interpolation weights from their
    general definition w_k = 1 / prod_{j != k} (s_k - s_j) (Eq. 2);
  * Lagrange polynomials in product form, L_k(y) = prod_{j != k} (y - s_j) / (s_k - s_j);
  * the approximated kernels of Eqs. (kernel-pc), (kernel-cp-v2) and
    (kernel-cc-v2) written as explicit matrices, so the whole BLDTT sum is
    sum over list entries of  [approximated G](x_i, y_j) q_j  with no upward
    or downward pass at all.
"""
from __future__ import annotations

import numpy as np


def cheb_points(n: int) -> np.ndarray:
    return np.cos(np.pi * np.arange(n + 1) / n)


def general_weights(s: np.ndarray) -> np.ndarray:
    """w_k = 1 / prod_{j != k} (s_k - s_j)."""
    m = s.shape[0]
    w = np.empty(m)
    for k in range(m):
        d = s[k] - np.delete(s, k)
        w[k] = 1.0 / np.prod(d)
    return w


def box_points(n: int, lo: float, hi: float) -> np.ndarray:
    return 0.5 * (lo + hi) + 0.5 * (hi - lo) * cheb_points(n)


def lagrange_product(s: np.ndarray, y: np.ndarray) -> np.ndarray:
    """L[a, k] = prod_{j != k} (y_a - s_j) / (s_k - s_j); exact at the nodes.

    A degenerate (zero-width) box has coincident nodes; the interpolant of a
    flat box is then the constant carried by node 0, as in the barycentric reading.
    """
    y = np.atleast_1d(np.asarray(y, dtype=np.float64))
    m = s.shape[0]
    if np.all(s == s[0]):
        out = np.zeros((y.shape[0], m))
        out[:, 0] = 1.0
        return out
    out = np.ones((y.shape[0], m))
    for k in range(m):
        for j in range(m):
            if j != k:
                out[:, k] *= (y - s[j]) / (s[k] - s[j])
    return out


def lagrange3(n: int, lo, hi, pts: np.ndarray) -> np.ndarray:
    """Tensor-product basis, L[a, k1 + (n+1) k2 + (n+1)^2 k3]."""
    Ls = [lagrange_product(box_points(n, lo[d], hi[d]), pts[:, d]) for d in range(3)]
    m = n + 1
    out = np.einsum("ai,aj,ak->akji", Ls[0], Ls[1], Ls[2]).reshape(pts.shape[0], m ** 3)
    return out


def grid3(n: int, lo, hi) -> np.ndarray:
    """Proxy points (rows) in flat order k1 + (n+1) k2 + (n+1)^2 k3."""
    s = [box_points(n, lo[d], hi[d]) for d in range(3)]
    k3, k2, k1 = np.meshgrid(np.arange(n + 1), np.arange(n + 1), np.arange(n + 1), indexing="ij")
    return np.stack([s[0][k1.ravel()], s[1][k2.ravel()], s[2][k3.ravel()]], axis=1)


def kernel_matrix(kernel: str, param: float, X: np.ndarray, Y: np.ndarray) -> np.ndarray:
    if kernel == "poly":
        return (1.0 + X @ Y.T) ** 2
    d = X[:, None, :] - Y[None, :, :]
    r2 = np.einsum("abk,abk->ab", d, d)
    r = np.sqrt(r2)
    with np.errstate(divide="ignore", invalid="ignore"):
        if kernel == "coulomb":
            G = 1.0 / r
        elif kernel == "yukawa":
            G = np.exp(-param * r) / r
        elif kernel == "oscillatory":
            G = np.sin(np.pi * r) / r
        elif kernel == "regcoulomb":
            G = 1.0 / np.sqrt(r2 + param * param)
        else:
            raise ValueError(kernel)
    G[r2 == 0.0] = 0.0
    return G


def direct_sum(tgt_xyz: np.ndarray, src_xyz: np.ndarray, q: np.ndarray, kernel="coulomb", param=0.0):
    return kernel_matrix(kernel, param, tgt_xyz, src_xyz) @ q


def explicit_bldtt(tgt_xyz, src_xyz, q, tree_t, tree_s, lists, n, kernel="coulomb", param=0.0):
    """sum over list entries of the approximated kernel matrix times the charges.

    lists[name] = (tcs, scs) with every approximation at degree n, or
    (tcs, scs, degs) with one degree per entry.

    PP: G(x_i, y_j); PC: sum_k G(x_i, s_k) L_k(y_j); CP: sum_l L_l(x_i) G(t_l, y_j);
    CC: sum_l sum_k L_l(x_i) G(t_l, s_k) L_k(y_j).  Trees give cluster membership
    (tree position ranges + permutation) and boxes; lists give (tc, sc) pairs.
    """
    phi = np.zeros(tgt_xyz.shape[0])

    def members(tree, c):
        b, cnt = tree["begin"][c], tree["count"][c]
        return tree["perm"][b:b + cnt]

    for name, entry in lists.items():
        tcs, scs = entry[0], entry[1]
        degs = entry[2] if len(entry) > 2 else [n] * len(tcs)
        for tc, sc, n in zip(tcs, scs, degs):
            n = int(n)
            ti = members(tree_t, tc)
            sj = members(tree_s, sc)
            X, Y = tgt_xyz[ti], src_xyz[sj]
            if name == "PP":
                A = kernel_matrix(kernel, param, X, Y)
            elif name == "PC":
                S = grid3(n, tree_s["lo"][sc], tree_s["hi"][sc])
                A = kernel_matrix(kernel, param, X, S) @ lagrange3(n, tree_s["lo"][sc], tree_s["hi"][sc], Y).T
            elif name == "CP":
                Tp = grid3(n, tree_t["lo"][tc], tree_t["hi"][tc])
                A = lagrange3(n, tree_t["lo"][tc], tree_t["hi"][tc], X) @ kernel_matrix(kernel, param, Tp, Y)
            else:
                Tp = grid3(n, tree_t["lo"][tc], tree_t["hi"][tc])
                S = grid3(n, tree_s["lo"][sc], tree_s["hi"][sc])
                A = (lagrange3(n, tree_t["lo"][tc], tree_t["hi"][tc], X) @ kernel_matrix(kernel, param, Tp, S)
                     @ lagrange3(n, tree_s["lo"][sc], tree_s["hi"][sc], Y).T)
            phi[ti] += A @ q[sj]
    return phi
