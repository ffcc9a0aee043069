"""GPU parity of the Vecchia/Matern preconditioner and the preconditioned solve.

Ordering and conditioning sets: bit-exact against the oracle's brute force
(including a lattice with many exactly tied distances).  Factor values:
1e-6 relative forward error (the blocks are ill-conditioned) plus a backward
error of the block solves at rounding level.  Solves: interpolant 1e-8
relative, w and beta within max(1e-8, 10x the two-direct-solver floor).
"""
import numpy as np
import pytest

from oracle import pcg as OP
from oracle import phs_dense as D
from oracle import vecchia as V
from paper_2608_11462_amd import native as N
from paper_2608_11462_amd import workloads as W
from tests.gpu_util import dev, host, rel

pytestmark = pytest.mark.gpu


def _oracle_factor(xy, k, m, nu, alpha, seed):
    c, rho, xi = D.normalize(xy, k)
    perm, rank = V.order(len(xy), seed)
    nbrs = V.ordered_knn(xi, perm, rank, m)
    cc, lams = V.factor(xi, nbrs, nu, alpha)
    return xi, perm, rank, nbrs, cc, lams


def _check_structure(xy, k, m, nu, alpha, seed, range_, units):
    n = len(xy)
    pl = N.Plan(dev(xy), k)
    pl.precond_build(m=m, nu=nu, range_=range_, range_units=units, seed=seed)
    rank_g, nbr_g, coef_g, diag_g = (host(t) for t in pl.precond_export(m))
    xi, perm, rank, nbrs, cc, lams = _oracle_factor(xy, k, m, nu, alpha, seed)
    np.testing.assert_array_equal(rank_g, rank)
    for j in range(n):
        s = nbrs[j]
        np.testing.assert_array_equal(nbr_g[j, :len(s)], s)
        assert np.all(nbr_g[j, len(s):] == -1)
    coef_ref = np.zeros((n, m))
    for j in range(n):
        coef_ref[j, :len(nbrs[j])] = -lams[j] / cc[j]
    ec = np.abs(coef_g - coef_ref).max() / np.abs(coef_ref).max()
    ed = np.abs(diag_g - 1.0 / cc).max() / np.abs(1.0 / cc).max()
    print(f"n={n} m={m} nu={nu}: coef err {ec:.2e}, diag err {ed:.2e}")
    # forward error is bounded by cond(K_ss) * eps: the blocks of a smooth
    # Matern kernel at close nodes are ill-conditioned, so compare loosely...
    assert ec <= 1e-6 and ed <= 1e-6
    # ...and check that the GPU's lambda solves its block equations to a
    # backward error at rounding level (eq. conditionals)
    worst = 0.0
    for j in W.sample_rows(3, n, 200):
        s = nbrs[j]
        if len(s) == 0:
            continue
        P = xi[s]
        Kss = V.matern(nu, alpha * np.sqrt(((P[:, None, :] - P[None, :, :]) ** 2).sum(-1)))
        ks = V.matern(nu, alpha * np.sqrt(((P - xi[j]) ** 2).sum(-1)))
        c_g = 1.0 / diag_g[j]
        lam_g = -coef_g[j, :len(s)] * c_g
        be = np.linalg.norm(Kss @ lam_g - ks) / (np.linalg.norm(Kss, 2) * np.linalg.norm(lam_g)
                                                 + np.linalg.norm(ks))
        worst = max(worst, be)
        assert abs(c_g * c_g - (1.0 - ks @ lam_g)) <= 1e-12
    print(f"worst backward error of the block solves {worst:.2e}")
    assert worst <= 1e-13
    return pl, xi, nbrs, cc, lams


def test_small_config_structure_and_factor():
    pr = W.small_tps()
    print(f"[case] small_tps vecchia n={pr.n}", flush=True)
    c, rho, xi = D.normalize(pr.xy, 2)
    alpha = 1.0 / (0.1 * rho)  # range 0.1 in user units
    pl, xi, nbrs, cc, lams = _check_structure(pr.xy, 2, 20, 1.5, alpha, 0, 0.1, N.PHS_RANGE_USER)
    # apply in caller order, against U~ U~^T r formed on the CPU from the
    # factor the GPU exported (tests the two gathers, not the factor values)
    rank_g, nbr_g, coef_g, diag_g = (host(t) for t in pl.precond_export(20))
    lam_g = [-coef_g[j, :len(nbrs[j])] / diag_g[j] for j in range(pr.n)]
    U = V.factor_matrix(pr.n, nbrs, 1.0 / diag_g, lam_g)
    r = W.rng_for(9).standard_normal(pr.n)
    z = host(pl.precond_apply(dev(r)))
    e = rel(z, V.apply(U, r))
    print(f"precond apply rel err {e:.2e}")
    assert e <= 1e-13


def test_paper_default_structure_nu1():
    """nu = 1 (Bessel K1 path), alpha = 0.35, m = 30 on [-1/4,1/4]^2."""
    xy = W.uniform_points(W.rng_for(41), 3000)
    print("[case] nu=1 default n=3000", flush=True)
    _check_structure(xy, 2, 30, 1.0, 0.35, 123, 0.0, N.PHS_RANGE_NORMALIZED)


def test_lattice_ties_bit_exact():
    """A regular lattice: many predecessors at exactly equal distance; ties are
    broken by rank."""
    g = np.arange(24) / 23.0
    xy = np.stack(np.meshgrid(g, g, indexing="ij"), axis=-1).reshape(-1, 2)
    print("[case] lattice ties n=576", flush=True)
    _check_structure(xy, 2, 12, 1.5, 5.0, 77, 0.2, N.PHS_RANGE_NORMALIZED)


@pytest.mark.parametrize("m", [1, 8, 16, 17, 32, 33, 63])
def test_conditioning_sets_bit_exact_list_sizes(m):
    """The search keeps each query's ordered list in blocks of 16 entries
    spread over 16 lanes (one, two or four blocks for m <= 16, 32, 63): every
    block count and the boundaries between them, on uniform nodes mixed with
    a lattice (many exactly tied distances, broken by rank), against the
    oracle's brute force (Sec. 3: the m nearest predecessors in the random
    ordering).  Only the ordering and the sets are compared."""
    g = np.arange(16) / 15.0
    lat = np.stack(np.meshgrid(g, g, indexing="ij"), axis=-1).reshape(-1, 2)
    xy = np.concatenate([W.uniform_points(W.rng_for(900 + m), 1500), 0.5 * lat + 0.25])
    n = len(xy)
    print(f"[case] conditioning sets m={m} n={n}", flush=True)
    pl = N.Plan(dev(xy), 2)
    pl.precond_build(m=m, nu=0.5, seed=m)
    rank_g, nbr_g, _, _ = (host(t) for t in pl.precond_export(m))
    pl.close()
    c, rho, xi = D.normalize(xy, 2)
    perm, rank = V.order(n, m)
    np.testing.assert_array_equal(rank_g, rank)
    nbrs = V.ordered_knn(xi, perm, rank, m)
    for j in range(n):
        s = nbrs[j]
        assert len(s) == min(m, rank[j])
        np.testing.assert_array_equal(nbr_g[j, :len(s)], s)
        assert np.all(nbr_g[j, len(s):] == -1)


@pytest.mark.parametrize("n,m", [(3, 30), (7, 30), (17, 16), (33, 63), (65, 63), (100, 63)])
def test_conditioning_sets_small_n(n, m):
    """Fewer nodes than (or about as many as) the set size: node j keeps all
    min(m, rank_j) predecessors, and queries end their search at the grid's
    edge rather than by the ring bound."""
    xy = W.uniform_points(W.rng_for(950 + n), n)
    print(f"[case] small conditioning sets n={n} m={m}", flush=True)
    pl = N.Plan(dev(xy), 2)
    pl.precond_build(m=m, nu=0.5, seed=n)
    rank_g, nbr_g, _, _ = (host(t) for t in pl.precond_export(m))
    pl.close()
    c, rho, xi = D.normalize(xy, 2)
    perm, rank = V.order(n, n)
    np.testing.assert_array_equal(rank_g, rank)
    nbrs = V.ordered_knn(xi, perm, rank, m)
    for j in range(n):
        s = nbrs[j]
        assert len(s) == min(m, rank[j])
        np.testing.assert_array_equal(nbr_g[j, :len(s)], s)
        assert np.all(nbr_g[j, len(s):] == -1)


def test_nu2_structure_k4():
    xy = W.uniform_points(W.rng_for(42), 1500)
    print("[case] k=4 nu=2 n=1500", flush=True)
    _check_structure(xy, 4, 50, 2.0, 2.0, 5, 0.0, N.PHS_RANGE_NORMALIZED)


def test_large_tps_ordering_and_sampled_knn_bit_exact():
    """The benchmark workload (n = 2^20, m = 30): the rank of every node, and the
    ordered neighbour lists of 1024 sampled nodes, bitwise against the brute
    force (the deeper rank-prefix grid levels of the search only occur here)."""
    pr = W.large_tps()
    print(f"[case] large_tps vecchia structure n={pr.n}", flush=True)
    m = 30
    pl = N.Plan(dev(pr.xy), 2, 1)
    pl.precond_build(m=m, nu=1.0, seed=0)
    rank_g, nbr_g, _, _ = pl.precond_export(m)
    rank_g, nbr_g = host(rank_g), host(nbr_g)
    pl.close()
    c, rho, xi = D.normalize(pr.xy, 2)
    perm, rank = V.order(pr.n, 0)
    np.testing.assert_array_equal(rank_g, rank)
    q = W.sample_rows(21, pr.n, 1024)
    # the earliest ranks (full conditioning, the coarse grid levels) as well
    q = np.unique(np.concatenate([q, perm[:64], perm[1000:1016]]))
    nbrs = V.ordered_knn(xi, perm, rank, m, q)
    for j, s in zip(q, nbrs):
        np.testing.assert_array_equal(nbr_g[j, :len(s)], s)
        assert np.all(nbr_g[j, len(s):] == -1)


@pytest.mark.parametrize("precision", [N.PHS_FP64, N.PHS_MIXED])
@pytest.mark.parametrize("pc", ["config", "paper"])
def test_small_config_solve(precision, pc):
    pr = W.small_tps()
    print(f"[case] small_tps solve precision={precision} pc={pc}", flush=True)
    ref = D.solve_complement(pr.xy, pr.f, 2, 1)
    bk = D.solve_bunch_kaufman(pr.xy, pr.f, 2, 1)
    pl = N.Plan(dev(pr.xy), 2, 1)
    if pc == "config":
        pl.precond_build(m=20, nu=1.5, range_=0.1, range_units=N.PHS_RANGE_USER, seed=0)
        c, rho, xi = D.normalize(pr.xy, 2)
        m, nu, alpha = 20, 1.5, 1.0 / (0.1 * rho)
    else:
        pl.precond_build(m=30, nu=1.0, seed=0)
        m, nu, alpha = 30, 1.0, 0.35
    # rtol 1e-12 so the weights (far more sensitive than the interpolant) are
    # resolved below 1e-8 of the direct solution
    w, beta, info = pl.solve(dev(pr.f), rtol=1e-12, precision=precision)
    w, beta = host(w), host(beta)
    dw = rel(bk["w"], ref["w"])
    ew, eb = rel(w, ref["w"]), rel(beta, ref["beta"])
    s_ref = D.interpolant(ref, 2, pr.targets)
    s = host(pl.eval(dev(w), dev(beta), dev(pr.targets)))
    es = np.abs(s - s_ref).max() / np.abs(s_ref).max()
    # oracle PCG with the same factor: expected iteration count
    xi, perm, rank, nbrs, cc, lams = _oracle_factor(pr.xy, 2, m, nu, alpha, 0)
    U = V.factor_matrix(pr.n, nbrs, cc, lams)
    M = D.kernel_matrix(2, xi, xi)
    Q = np.linalg.qr(D.poly_block(xi, 1))[0]
    _, it_ref, _ = OP.pcg_projected(lambda v: M @ v, lambda r: V.apply(U, r), Q, pr.f, 1,
                                    rtol=1e-12)
    print(f"iters gpu={info.iters} (outer {info.outer_refinements}) oracle={it_ref} "
          f"resid={info.rel_residual:.2e} w {ew:.2e} beta {eb:.2e} interp {es:.2e} "
          f"floor {dw:.2e}")
    assert ew <= max(1e-8, 10 * dw)
    assert eb <= max(1e-8, 10 * rel(bk["beta"], ref["beta"]))
    assert es <= 1e-8
    if precision == N.PHS_FP64:
        assert abs(info.iters - it_ref) <= 2
