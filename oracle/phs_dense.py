"""Dense FP64 definition of PHS interpolation (oracle; test infrastructure only).

Everything here follows Sec. 1-2 of the paper directly:

* the interpolant  f(x) = sum_s beta_s P_s(x) + sum_j w_j phi(|x_j - x|)   (eq. phs_interp)
* the basis        phi(r) = r^k (k odd),  r^k log r (k even)               (eq. phs_fun)
* the saddle system [M B; B^T 0][w; beta] = [f; 0]                         (eq. phs_linsys)
* its solution on the complement of span(B): Q_perp^T M Q_perp u = Q_perp^T f,
  w = Q_perp u,  R beta = Q^T (f - M w)                                    (eq. phs_linsys_solve)
* the normalisation of the points (scale and translation, eq. M_rho and the
  tuned domains of Sec. 2.2).

Readings taken where the text is garbled or silent (each is listed in the
design notes):

* The polynomial block B is n x S with B[j, s] = P_s(x_j) and the constraint is
  B^T w = 0 (the printed system shows B in both off-diagonal blocks).
* The polynomial space is all monomials of total degree <= d; the minimal d is
  ceil(k/2)-1 for odd k and k/2 for even k (conditional positive definiteness
  order of the PHS kernels).  Monomials are ordered by total degree, then by
  descending power of the first coordinate: 1, x, y, x^2, xy, y^2, ...
* Q_perp^T M Q_perp is definite but its sign depends on k: it is positive
  definite when k mod 4 is 2 or 3 and negative definite otherwise.  The
  factorisation is applied to sign_k * A.
* Points are normalised as xi = (x - c) * rho, with c the bounding-box centre,
  rho = h_k / half, half = half the larger bounding-box extent, and h_k = 1/4
  (k=2), 1 (k=4), 1/2 (odd k), 1 (even k >= 6).  w and beta are reported in
  these normalised coordinates.
* Pairs at distance zero contribute phi(0) = 0 (the diagonal of M and of the
  core log matrix is zero).
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg as sla


# ----------------------------------------------------------------- basics

def h_domain(k: int) -> float:
    """Half-width of the normalised domain [-h, h]^2 (Sec. 2.2 tuning: TPS on
    [-1/4,1/4]^2, k=4 on [-1,1]^2; odd k reading: 1/2)."""
    if k == 2:
        return 0.25
    if k % 2 == 1:
        return 0.5
    return 1.0


def d_min(k: int) -> int:
    """Minimal total degree of the polynomial block for order k."""
    return (k + 1) // 2 - 1 if k % 2 == 1 else k // 2


def sign_k(k: int) -> int:
    """+1 if Q_perp^T M Q_perp is positive definite, -1 if negative definite."""
    return 1 if (k % 4) in (2, 3) else -1


def normalize(xy: np.ndarray, k: int):
    """Return (c, rho, xi).  Operation order: c = (min+max)*0.5,
    half = max(extent_x, extent_y)*0.5, rho = h/half, xi = (x-c)*rho."""
    xy = np.asarray(xy, dtype=np.float64)
    mn = xy.min(axis=0)
    mx = xy.max(axis=0)
    c = (mn + mx) * 0.5
    ext = mx - mn
    half = max(ext[0], ext[1]) * 0.5
    if not half > 0.0:
        raise ValueError("degenerate point set (zero extent)")
    rho = h_domain(k) / half
    xi = (xy - c) * rho
    return c, rho, xi


def monomials(d: int):
    """Exponent pairs (a, b) of x^a y^b, total degree 0..d, descending a."""
    out = []
    for t in range(d + 1):
        for a in range(t, -1, -1):
            out.append((a, t - a))
    return out


def poly_block(xi: np.ndarray, d: int) -> np.ndarray:
    """B[j, s] = P_s(xi_j) for the monomials of total degree <= d."""
    cols = [xi[:, 0] ** a * xi[:, 1] ** b for (a, b) in monomials(d)]
    return np.stack(cols, axis=1)


def phi(k: int, r: np.ndarray) -> np.ndarray:
    """eq. phs_fun with phi(0) = 0."""
    r = np.asarray(r, dtype=np.float64)
    out = np.zeros_like(r)
    nz = r > 0.0
    rk = r[nz] ** k
    if k % 2 == 1:
        out[nz] = rk
    else:
        out[nz] = rk * np.log(r[nz])
    return out


def pair_dist(X: np.ndarray, Y: np.ndarray) -> np.ndarray:
    dx = X[:, None, 0] - Y[None, :, 0]
    dy = X[:, None, 1] - Y[None, :, 1]
    return np.sqrt(dx * dx + dy * dy)


def kernel_matrix(k: int, X: np.ndarray, Y: np.ndarray) -> np.ndarray:
    """M[i, j] = phi(|X_i - Y_j|)."""
    return phi(k, pair_dist(X, Y))


# ----------------------------------------------------------------- solvers

class Unisolvent(Exception):
    """The polynomial block is rank deficient on the given points."""


def _qr_split(B: np.ndarray):
    Qf, Rf = np.linalg.qr(B, mode="complete")
    S = B.shape[1]
    R = Rf[:S, :S]
    diag = np.abs(np.diag(R))
    if diag.min() <= 1e-12 * diag.max():
        raise Unisolvent("polynomial block is not of full column rank")
    return Qf[:, :S], Qf[:, S:], R


def solve_complement_xi(xi: np.ndarray, f, k: int, d: int):
    """eq. phs_linsys_solve on given (already normalised) coordinates.
    Returns (w, beta, Q, R)."""
    B = poly_block(xi, d)
    Q, Qp, R = _qr_split(B)
    M = kernel_matrix(k, xi, xi)
    s = sign_k(k)
    f = np.asarray(f, dtype=np.float64)
    if Qp.shape[1] == 0:          # n == S: the polynomial interpolates alone
        w = np.zeros_like(f)
    else:
        A = s * (Qp.T @ M @ Qp)
        A = 0.5 * (A + A.T)
        L = sla.cho_factor(A, lower=True)
        u = sla.cho_solve(L, s * (Qp.T @ f))
        w = Qp @ u
    beta = sla.solve_triangular(R, Q.T @ (f - M @ w), lower=False)
    return w, beta, Q, R


def solve_complement(xy, f, k: int, d: int = -1):
    """Direct solution following eq. phs_linsys_solve on the normalised nodes.

    Returns dict(w, beta, c, rho, xi, Q, R, degree).  f may be (n,) or (n, nrhs).
    """
    if d < 0:
        d = d_min(k)
    c, rho, xi = normalize(xy, k)
    w, beta, Q, R = solve_complement_xi(xi, f, k, d)
    return dict(w=w, beta=beta, c=c, rho=rho, xi=xi, Q=Q, R=R, degree=d)


def solve_bunch_kaufman(xy, f, k: int, d: int = -1):
    """The paper's exact baseline: a symmetric-indefinite (Bunch-Kaufman)
    factorisation of the full (n+S) x (n+S) saddle matrix (Sec. 1)."""
    if d < 0:
        d = d_min(k)
    c, rho, xi = normalize(xy, k)
    B = poly_block(xi, d)
    n, S = B.shape
    M = kernel_matrix(k, xi, xi)
    A = np.zeros((n + S, n + S))
    A[:n, :n] = M
    A[:n, n:] = B
    A[n:, :n] = B.T
    f = np.asarray(f, dtype=np.float64)
    rhs = np.zeros((n + S,) + f.shape[1:])
    rhs[:n] = f
    lu, piv, _ = sla.lapack.dsytrf(A, lower=0)
    sol, info = sla.lapack.dsytrs(lu, piv, rhs, lower=0)
    if info != 0:
        raise RuntimeError("dsytrs failed")
    return dict(w=sol[:n], beta=sol[n:], c=c, rho=rho, xi=xi, degree=d)


def interpolant(sol: dict, k: int, targets: np.ndarray) -> np.ndarray:
    """Evaluate eq. phs_interp at user-coordinate targets."""
    xt = (np.asarray(targets, dtype=np.float64) - sol["c"]) * sol["rho"]
    P = poly_block(xt, sol["degree"])
    Kt = kernel_matrix(k, xt, sol["xi"])
    return P @ sol["beta"] + Kt @ sol["w"]


# ----------------------------------------------------------------- matvec

def matvec_dense(k: int, xi: np.ndarray, v: np.ndarray) -> np.ndarray:
    """y = M v with the dense kernel matrix."""
    return kernel_matrix(k, xi, xi) @ v


def _compensated_row_sums(block_fn, rows_count: int, n_cols: int, col_chunk: int) -> np.ndarray:
    """Sum each row of a (rows_count x n_cols) implicit matrix: pairwise sums
    over column chunks, then an exactly rounded sum (math.fsum) of the chunk
    sums per row."""
    parts = []
    for c0 in range(0, n_cols, col_chunk):
        parts.append(block_fn(c0, min(n_cols, c0 + col_chunk)).sum(axis=1))
    parts = np.stack(parts, axis=1)
    return np.array([math.fsum(p) for p in parts])


def matvec_rows(k: int, xi: np.ndarray, v: np.ndarray, rows: np.ndarray,
                row_chunk: int = 64, col_chunk: int = 1 << 16) -> np.ndarray:
    """(M v)[rows] by direct summation over all n sources (r=0 pairs give 0)."""
    rows = np.asarray(rows)
    out = np.empty(len(rows))
    n = xi.shape[0]
    for r0 in range(0, len(rows), row_chunk):
        rr = rows[r0:r0 + row_chunk]
        X = xi[rr]

        def blk(c0, c1, X=X):
            return kernel_matrix(k, X, xi[c0:c1]) * v[None, c0:c1]
        out[r0:r0 + len(rr)] = _compensated_row_sums(blk, len(rr), n, col_chunk)
    return out


def eval_points(k: int, xi_nodes: np.ndarray, w: np.ndarray, beta: np.ndarray, degree: int,
                xi_targets: np.ndarray, row_chunk: int = 64, col_chunk: int = 1 << 16) -> np.ndarray:
    """eq. phs_interp at normalised targets by direct summation (large n)."""
    out = np.empty(len(xi_targets))
    n = xi_nodes.shape[0]
    P = poly_block(xi_targets, degree)
    for r0 in range(0, len(xi_targets), row_chunk):
        X = xi_targets[r0:r0 + row_chunk]

        def blk(c0, c1, X=X):
            return kernel_matrix(k, X, xi_nodes[c0:c1]) * w[None, c0:c1]
        out[r0:r0 + len(X)] = _compensated_row_sums(blk, len(X), n, col_chunk)
    return out + P @ beta


# ----------------------------------------------------------------- Hadamard

def power_factors(q: int, X: np.ndarray, Y: np.ndarray):
    """Separable factors of the even-power distance matrix [|x_i - y_j|^{2q}].

    Expands (a + b - 2 x.y)^q with a = |x|^2, b = |y|^2 by the multinomial
    theorem and (x.y)^l by the binomial theorem (eq. norm_sep).  Returns
    (U, V) with [|x_i - y_j|^{2q}] = U V^T.  The expansion is exact but not of
    minimal rank.
    """
    a = X[:, 0] ** 2 + X[:, 1] ** 2
    b = Y[:, 0] ** 2 + Y[:, 1] ** 2
    ucols, vcols = [], []
    for i in range(q + 1):
        for j in range(q + 1 - i):
            l = q - i - j
            coef = math.factorial(q) / (math.factorial(i) * math.factorial(j) * math.factorial(l))
            coef *= (-2.0) ** l
            for t in range(l + 1):
                ct = coef * math.comb(l, t)
                ucols.append(ct * a ** i * X[:, 0] ** t * X[:, 1] ** (l - t))
                vcols.append(b ** j * Y[:, 0] ** t * Y[:, 1] ** (l - t))
    return np.stack(ucols, axis=1), np.stack(vcols, axis=1)


def core_matrix(kind: str, X: np.ndarray, Y: np.ndarray) -> np.ndarray:
    """The core kernel: log r (kind='log') or r (kind='dist'), zero at r=0."""
    r = pair_dist(X, Y)
    if kind == "log":
        out = np.zeros_like(r)
        nz = r > 0
        out[nz] = np.log(r[nz])
        return out
    return r


def hadamard_matvec(k: int, xi: np.ndarray, t: np.ndarray) -> np.ndarray:
    """eq. matvec_hadamard: M t = sum_l D_{u_l} M_core D_{v_l} t, with
    M = M_core o [r^{2q}], q = floor(k/2), core log for even k and r for odd k."""
    q = k // 2
    kind = "log" if k % 2 == 0 else "dist"
    U, V = power_factors(q, xi, xi)
    C = core_matrix(kind, xi, xi)
    y = np.zeros_like(t, dtype=np.float64)
    for l in range(U.shape[1]):
        y += U[:, l] * (C @ (V[:, l] * t))
    return y


# ----------------------------------------------------------------- tree

def leaf_order(xi: np.ndarray, h: float, L: int):
    """CPU reference of the quadtree leaf assignment: cell q = floor((xi + h) *
    2^L / (2h)) clamped to [0, 2^L), row-major key q_y * 2^L + q_x, nodes
    sorted stably by key (ties by caller index).  Returns (order, keys_sorted)."""
    G = 1 << L
    scale = G / (2.0 * h)
    q = np.floor((xi + h) * scale).astype(np.int64)
    q = np.clip(q, 0, G - 1)
    key = q[:, 1] * G + q[:, 0]
    order = np.argsort(key, kind="stable")
    return order, key[order]
