"""GPU parity of the hot path against the dense FP64 oracle (through the C ABI).

Inputs: the seeded small thin-plate workload (n=2000 uniform points, k=2,
linear block) and small variants for other orders.  Tolerances:
FP64 matvec relative 2-norm error <= 1e-10; tree order bit-exact; solve:
interpolant <= 1e-8 relative (max norm), w and beta within max(1e-8, 10x the
disagreement of two independent direct solvers).
"""
import numpy as np
import pytest
import torch

from oracle import phs_dense as D
from paper_2608_11462_amd import native as N
from paper_2608_11462_amd import workloads as W
from tests.gpu_util import dev, host, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def small():
    pr = W.small_tps()
    print(f"[case] small_tps n={pr.n}", flush=True)
    return pr


def _plan(pr, k=None, degree=None, **kw):
    return N.Plan(dev(pr.xy), k if k is not None else pr.k,
                  degree if degree is not None else pr.degree, **kw)


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_normalisation_and_tree_bit_exact(small, k):
    pl = _plan(small, k=k, degree=-1)
    c, rho, xi = D.normalize(small.xy, k)
    assert pl.center == (c[0], c[1])
    assert pl.scale == rho
    order, leaf = pl.tree()
    assert pl.tree_half_width >= D.h_domain(k)
    order_ref, keys_ref = D.leaf_order(xi, pl.tree_half_width, pl.leaf_level)
    np.testing.assert_array_equal(host(order), order_ref)
    np.testing.assert_array_equal(host(leaf), keys_ref)


@pytest.mark.parametrize("name", ["large_tps", "odd_clustered"])
def test_tree_bit_exact_full_size(name):
    """Every node's tree position and leaf key at the full sizes (n = 2^20
    uniform, k = 2, L = 7; n = 1e5 clustered, k = 3, deepened), bitwise against
    the CPU reference, and the leaf level against the deepening rule (the
    leaf level is round(log4(n / s)) clamped to 2..10, deepened while a leaf
    holds more than 16 s nodes; s = 40 for even k, 64 for odd k)."""
    pr = getattr(W, name)()
    print(f"[case] tree {name} n={pr.n}", flush=True)
    pl = N.Plan(dev(pr.xy), pr.k, pr.degree)
    c, rho, xi = D.normalize(pr.xy, pr.k)
    order, leaf = pl.tree()
    order_ref, keys_ref = D.leaf_order(xi, pl.tree_half_width, pl.leaf_level)
    np.testing.assert_array_equal(host(order), order_ref)
    np.testing.assert_array_equal(host(leaf), keys_ref)
    s = 40 if pr.k % 2 == 0 else 64
    L0 = min(10, max(2, int(round(np.log(pr.n / s) / np.log(4.0)))))
    L = pl.leaf_level
    assert L >= L0
    if L < 10:
        assert np.bincount(keys_ref).max() <= 16 * s
    if L > L0:
        _, keys_up = D.leaf_order(xi, pl.tree_half_width, L - 1)
        assert np.bincount(keys_up).max() > 16 * s
    pl.close()


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_matvec_fp64_parity(small, k):
    pl = _plan(small, k=k, degree=-1)
    c, rho, xi = D.normalize(small.xy, k)
    rng = W.rng_for(100 + k)
    v = rng.standard_normal(small.n)
    y_ref = D.matvec_dense(k, xi, v)
    y = host(pl.matvec(dev(v)))
    e = rel(y, y_ref)
    print(f"k={k} L={pl.leaf_level} p={pl.order} fp64 matvec rel err {e:.3e}")
    assert e <= 1e-10
    # projected input (the vectors PCG applies M to)
    B = D.poly_block(xi, D.d_min(k))
    Q, _ = np.linalg.qr(B)
    vp = v - Q @ (Q.T @ v)
    e2 = rel(host(pl.matvec(dev(vp))), D.matvec_dense(k, xi, vp))
    print(f"k={k} projected fp64 matvec rel err {e2:.3e}")
    assert e2 <= 1e-10


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_matvec_mixed_reported(small, k):
    pl = _plan(small, k=k, degree=-1)
    c, rho, xi = D.normalize(small.xy, k)
    v = W.rng_for(200 + k).standard_normal(small.n)
    y_ref = D.matvec_dense(k, xi, v)
    e = rel(host(pl.matvec(dev(v), precision=N.PHS_MIXED)), y_ref)
    print(f"k={k} mixed (FP32) matvec rel err {e:.3e}")
    assert e <= 1e-4


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_matvec_near32(small, k):
    """FP64 far field with an FP32 near field: the near-field entries are small,
    so the matvec stays close to FP64 accuracy."""
    pl = _plan(small, k=k, degree=-1)
    c, rho, xi = D.normalize(small.xy, k)
    v = W.rng_for(300 + k).standard_normal(small.n)
    y_ref = D.matvec_dense(k, xi, v)
    e = rel(host(pl.matvec(dev(v), precision=N.PHS_NEAR32)), y_ref)
    print(f"k={k} near32 matvec rel err {e:.3e}")
    assert e <= 1e-6


def test_matvec_multi_rhs(small):
    pl = _plan(small)
    c, rho, xi = D.normalize(small.xy, 2)
    V = W.rng_for(7).standard_normal((small.n, 3))
    Y = host(pl.matvec(dev(V)))
    Y_ref = D.matvec_dense(2, xi, V)
    assert rel(Y, Y_ref) <= 1e-10


def test_solve_identity_preconditioner():
    # unpreconditioned CG needs many iterations on the TPS system: keep n small
    small = W.small_tps(n=500)
    pl = _plan(small)
    ref = D.solve_complement(small.xy, small.f, 2, 1)
    bk = D.solve_bunch_kaufman(small.xy, small.f, 2, 1)
    dw = rel(ref["w"], bk["w"])
    # unpreconditioned, the weights carry kappa * rtol: a tight rtol
    w, beta, info = pl.solve(dev(small.f), rtol=1e-12, maxit=20000)
    w, beta = host(w), host(beta)
    ew, eb = rel(w, ref["w"]), rel(beta, ref["beta"])
    print(f"identity-PCG iters={info.iters} resid={info.rel_residual:.2e} "
          f"w err {ew:.2e} beta err {eb:.2e} (direct-solver floor {dw:.2e})")
    # floor-aware: two direct solvers already disagree on w by dw
    assert ew <= max(1e-8, 10 * dw)
    assert eb <= max(1e-8, 10 * rel(bk["beta"], ref["beta"]))
    s_ref = D.interpolant(ref, 2, small.targets)
    s = host(pl.eval(dev(w), dev(beta), dev(small.targets)))
    es = np.abs(s - s_ref).max() / np.abs(s_ref).max()
    print(f"interpolant at targets max rel err {es:.2e}")
    assert es <= 1e-8


# Expansion order P set explicitly: the FP64 orders with matrix-core M2L and
# row-segment M2M/L2L (15, 23, 27, 31) and one on the generic vector path
# (20), against the dense matvec.  Bounds at about 100x the measured error
# (k = 2: 9.8e-10 at P = 15 down to 1.7e-15 at P = 31); an error in a
# kernel's tiling would show up at order one.
_LOG_P_TOL = {15: 1e-7, 20: 1e-9, 23: 1e-10, 27: 3e-12, 31: 3e-13, 40: 1e-14, 63: 1e-14}


# Orders above 31 take one leaf per wavefront in P2M (smaller point chunks in
# LDS) and the vector-unit M2M/M2L/L2L.
@pytest.mark.parametrize("k", [2, 4])
@pytest.mark.parametrize("p", [15, 20, 23, 27, 31, 40, 63])
def test_matvec_every_order(k, p):
    rng = W.rng_for(330 + k)
    xy = W.uniform_points(rng, 12000)
    print(f"[case] k={k} P={p}", flush=True)
    pl = N.Plan(dev(xy), k, leaf_size=16, expansion_order=p)
    assert pl.order == p
    c, rho, xi = D.normalize(xy, k)
    v = W.rng_for(9).standard_normal(len(xy))
    y_ref = D.matvec_dense(k, xi, v)
    e = rel(host(pl.matvec(dev(v))), y_ref)
    print(f"k={k} P={p} L={pl.leaf_level}: fp64 matvec rel err {e:.2e}")
    assert e <= _LOG_P_TOL[p]


# Seven levels (L2L into level 7 by row segments) for the segment orders other
# than the default: rows sampled from the dense matvec.
@pytest.mark.parametrize("p", [15, 23, 31])
def test_matvec_deep_tree_orders(p):
    k = 2
    rng = W.rng_for(340)
    xy = W.uniform_points(rng, 200000)
    print(f"[case] deep tree k={k} P={p} n={len(xy)}", flush=True)
    pl = N.Plan(dev(xy), k, leaf_size=8, expansion_order=p)
    assert pl.leaf_level >= 7
    c, rho, xi = D.normalize(xy, k)
    v = W.rng_for(10).standard_normal(len(xy))
    y = host(pl.matvec(dev(v)))
    rows = np.sort(W.rng_for(11).choice(len(xy), 512, replace=False))
    y_ref = np.concatenate([D.kernel_matrix(k, xi[rows[i:i + 64]], xi) @ v
                            for i in range(0, len(rows), 64)])
    e = np.linalg.norm(y[rows] - y_ref) / np.linalg.norm(y_ref)
    print(f"k={k} P={p} L={pl.leaf_level}: sampled fp64 matvec rel err {e:.2e}")
    assert e <= _LOG_P_TOL[p]
