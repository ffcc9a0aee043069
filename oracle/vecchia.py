"""Vecchia / Matern sparse inverse-Cholesky preconditioner (oracle; test
infrastructure only).  Follows Sec. 2.2: the Matern covariance, the
conditionals of eq. conditionals with conditioning sets sigma(j), and the
sparse "reverse" inverse-Cholesky factor of Fig. vecchia_chol, whose column j
holds 1/c on the diagonal and -lambda/c at the rows sigma(j).

Readings (the paper leaves these open):

* Ordering: the random permutation of Sec. 3 is made reproducible as
  "sort the points by (splitmix64(seed XOR i), i)", i the caller's index.
  splitmix64 is Steele, Lea and Flood's finaliser (add 0x9E3779B97F4A7C15,
  then two xor-shift-multiply rounds and a final xor-shift).
* sigma(j) = the m points of smaller rank with the smallest (d^2, rank), where
  d^2 = dx*dx + dy*dy in FP64 (each product rounded, then the sum) on the
  normalised coordinates.  A point with fewer than m predecessors conditions on
  all of them ("full conditioning" of Sec. 3).  sigma(j) is listed in that
  ascending (d^2, rank) order.
* Matern: K(r) = 2^(1-nu)/Gamma(nu) (alpha r)^nu K_nu(alpha r), K(0) = 1,
  alpha the inverse range (Sec. 2.2 uses alpha in this role).
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.special as ss

_M64 = (1 << 64) - 1


def splitmix64(x: int) -> int:
    """The splitmix64 output function applied to state x (one step)."""
    z = (x + 0x9E3779B97F4A7C15) & _M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
    return z ^ (z >> 31)


def splitmix64_np(x: np.ndarray) -> np.ndarray:
    """Vectorised splitmix64 on uint64 arrays (wrap-around arithmetic)."""
    with np.errstate(over="ignore"):
        z = x.astype(np.uint64) + np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def order(n: int, seed: int):
    """Return (perm, rank): perm[t] = caller index of rank t; rank = inverse."""
    idx = np.arange(n, dtype=np.uint64)
    keys = splitmix64_np(idx ^ np.uint64(seed & _M64))
    perm = np.lexsort((idx, keys)).astype(np.int64)
    rank = np.empty(n, dtype=np.int64)
    rank[perm] = np.arange(n)
    return perm, rank


def _d2(xi: np.ndarray, cand: np.ndarray, j: int) -> np.ndarray:
    dx = xi[cand, 0] - xi[j, 0]
    dy = xi[cand, 1] - xi[j, 1]
    return dx * dx + dy * dy


def ordered_knn(xi: np.ndarray, perm: np.ndarray, rank: np.ndarray, m: int,
                queries=None):
    """Brute force: for each query point j, the min(m, rank_j) predecessors with
    the smallest (d^2, rank).  Returns a list of int64 arrays (caller indices),
    one per query (all points when queries is None)."""
    n = xi.shape[0]
    if queries is None:
        queries = np.arange(n)
    out = []
    for j in queries:
        t = rank[j]
        prior = perm[:t]
        if t == 0:
            out.append(np.zeros(0, dtype=np.int64))
            continue
        d2 = _d2(xi, prior, j)
        if t > m:
            # only candidates no farther than the m-th smallest distance can be
            # chosen; all of them (ties included) go on to the sort
            thr = np.partition(d2, m - 1)[m - 1]
            keep = d2 <= thr
            prior, d2 = prior[keep], d2[keep]
        o = np.lexsort((rank[prior], d2))[:m]
        out.append(prior[o])
    return out


def matern(nu: float, x: np.ndarray) -> np.ndarray:
    """Normalised Matern correlation 2^(1-nu)/Gamma(nu) x^nu K_nu(x), value 1 at 0."""
    x = np.asarray(x, dtype=np.float64)
    out = np.ones_like(x)
    nz = x > 0
    xn = x[nz]
    out[nz] = (2.0 ** (1.0 - nu) / math.gamma(nu)) * xn ** nu * ss.kv(nu, xn)
    return out


def factor(xi: np.ndarray, nbrs, nu: float, alpha: float):
    """Per point j: lambda_j = K_ss^{-1} k_sj and c_j^2 = K(0) - k_sj^T lambda_j
    (eq. conditionals restricted to sigma(j)).  Returns (c, lams)."""
    n = xi.shape[0]
    c = np.empty(n)
    lams = []
    for j in range(n):
        s = nbrs[j]
        if len(s) == 0:
            c[j] = 1.0
            lams.append(np.zeros(0))
            continue
        P = xi[s]
        Kss = matern(nu, alpha * np.sqrt(_pd2(P, P)))
        dv = P - xi[j]
        ks = matern(nu, alpha * np.sqrt(dv[:, 0] * dv[:, 0] + dv[:, 1] * dv[:, 1]))
        L = sla.cho_factor(Kss, lower=True)
        lam = sla.cho_solve(L, ks)
        c2 = 1.0 - ks @ lam
        c[j] = math.sqrt(c2)
        lams.append(lam)
    return c, lams


def _pd2(X, Y):
    dx = X[:, None, 0] - Y[None, :, 0]
    dy = X[:, None, 1] - Y[None, :, 1]
    return dx * dx + dy * dy


def factor_matrix(n: int, nbrs, c: np.ndarray, lams) -> sp.csc_matrix:
    """U~ in caller index space: U[j,j] = 1/c_j, U[sigma(j), j] = -lambda/c_j
    (Fig. vecchia_chol).  Sigma^{-1} ~= U U^T."""
    rows, cols, vals = [], [], []
    for j in range(n):
        rows.append(j)
        cols.append(j)
        vals.append(1.0 / c[j])
        s = nbrs[j]
        rows.extend(s.tolist())
        cols.extend([j] * len(s))
        vals.extend((-lams[j] / c[j]).tolist())
    return sp.csc_matrix((vals, (rows, cols)), shape=(n, n))


def apply(U: sp.csc_matrix, r: np.ndarray) -> np.ndarray:
    """z = U (U^T r)."""
    return U @ (U.T @ r)


def covariance(xi: np.ndarray, nu: float, alpha: float) -> np.ndarray:
    """Dense Matern covariance Sigma on normalised points."""
    return matern(nu, alpha * np.sqrt(_pd2(xi, xi)))
