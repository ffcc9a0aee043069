"""Odd orders (distance-kernel FMM) against the dense oracle: k = 1 and 3,
uniform and clustered nodes, several leaf depths so the far field is
exercised on more than one level.  Solves are gated on the interpolant and
the node residual (1e-8); weights, which the odd-order systems determine only
to their conditioning, are compared against the direct-solver floor."""
import numpy as np
import pytest

from oracle import phs_dense as D
from paper_2608_11462_amd import native as N
from paper_2608_11462_amd import workloads as W
from tests.gpu_util import dev, host, rel

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("k", [1, 3])
@pytest.mark.parametrize("geom", ["uniform", "clustered"])
@pytest.mark.parametrize("leaf", [16, 64])
def test_odd_matvec_parity(k, geom, leaf):
    rng = W.rng_for(300 + k)
    xy = W.uniform_points(rng, 4000) if geom == "uniform" else W.clustered_points(rng, 4000)
    print(f"[case] k={k} {geom} leaf={leaf}", flush=True)
    pl = N.Plan(dev(xy), k, leaf_size=leaf)
    c, rho, xi = D.normalize(xy, k)
    v = W.rng_for(7).standard_normal(len(xy))
    y_ref = D.matvec_dense(k, xi, v)
    e = rel(host(pl.matvec(dev(v))), y_ref)
    em = rel(host(pl.matvec(dev(v), N.PHS_MIXED)), y_ref)
    print(f"k={k} {geom} L={pl.leaf_level} Q={pl.order}: fp64 {e:.2e} mixed {em:.2e}")
    assert e <= 1e-10
    assert em <= 1e-4


@pytest.mark.parametrize("k,d", [(1, 0), (3, 1), (3, 2)])
def test_odd_solve_and_eval(k, d):
    rng = W.rng_for(310 + k + d)
    xy = W.clustered_points(rng, 2500)
    f = W.bump_field(rng)(xy)
    tg = np.concatenate([W.uniform_points(rng, 300),
                         W.uniform_points(rng, 20) * 3.0 - 1.0])  # some outside the box
    print(f"[case] odd solve k={k} d={d}", flush=True)
    ref = D.solve_complement(xy, f, k, d)
    bk = D.solve_bunch_kaufman(xy, f, k, d)
    pl = N.Plan(dev(xy), k, d)
    pl.precond_build(m=50, nu=k / 2.0, seed=3)
    w, beta, info = pl.solve(dev(f), rtol=1e-12)
    w, beta = host(w), host(beta)
    s = host(pl.eval(dev(w), dev(beta), dev(tg)))
    s_ref = D.interpolant(ref, k, tg)
    es = np.abs(s - s_ref).max() / np.abs(s_ref).max()
    ew, dw = rel(w, ref["w"]), rel(bk["w"], ref["w"])
    xi = ref["xi"]
    res = D.kernel_matrix(k, xi, xi) @ w + D.poly_block(xi, d) @ beta - f
    er = np.abs(res).max() / np.abs(f).max()
    print(f"k={k} d={d} iters={info.iters} resid={info.rel_residual:.2e} w {ew:.2e} "
          f"(floor {dw:.2e}) interp {es:.2e} node residual {er:.2e}")
    assert es <= 1e-8
    assert er <= 1e-8
    # floor-aware: two direct solvers already disagree on w by dw
    assert ew <= max(1e-8, 10 * dw)


# Chebyshev order Q per axis set explicitly: every FP64 M2L tile shape
# (QQ = 64, 100, 144, 196, 256 output rows, the last row tile partly padded
# for QQ = 100 and 196) against the dense matvec.  The bounds follow the
# interpolation error (measured 1e-8 at Q = 8 down to 1.3e-14 at Q = 16, k = 1),
# with a margin of about 100; an error in
# the tiling would show up at order one.
_ODD_Q_TOL = {8: 1e-6, 10: 3e-8, 12: 1e-9, 14: 3e-11, 16: 1e-12}


@pytest.mark.parametrize("k", [1, 3])
@pytest.mark.parametrize("q", [8, 10, 12, 14, 16])
def test_odd_matvec_every_order(k, q):
    rng = W.rng_for(320 + k)
    xy = W.uniform_points(rng, 3000)
    print(f"[case] k={k} Q={q}", flush=True)
    pl = N.Plan(dev(xy), k, leaf_size=16, expansion_order=q)
    assert pl.order == q
    c, rho, xi = D.normalize(xy, k)
    v = W.rng_for(8).standard_normal(len(xy))
    y_ref = D.matvec_dense(k, xi, v)
    e = rel(host(pl.matvec(dev(v))), y_ref)
    print(f"k={k} Q={q} L={pl.leaf_level}: fp64 matvec rel err {e:.2e}")
    assert e <= _ODD_Q_TOL[q]
