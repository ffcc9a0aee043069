"""Full-size workloads, checked on sampled outputs by FP64 direct summation
(the dense oracle cannot form these matrices; the sampled sums run in the
oracle's plain-C direct summation).

* odd_clustered: n = 100000 (70% uniform + 30% in 10 Gaussian clusters), k = 3,
  quadratic block, Vecchia m = 50, nu = 1.5, alpha = 3 (the k = 3 default).
* large_tps: n = 2^20 uniform, k = 2, linear block, Vecchia m = 30, nu = 1,
  alpha = 0.35 (the benchmark configuration).

Gates, on 4096 seeded sampled rows / targets:
  matvec (FP64)                       <= 1e-10 relative 2-norm on the rows;
  the solver's FP64 exit residual     <= 1e-8 (over all nodes);
  node residual RMS(f - M w - B beta) / RMS(f) by direct summation <= 1e-8;
  evaluation at the targets vs direct summation with the same (w, beta)
                                       <= 1e-10 relative.
The interpolant is a sum of large alternating w_j phi terms (an FMM error of
~2e-14 relative to sum |w_j phi| shows up as ~1e-10 relative to max |s|),
which is why target evaluation uses the tighter FP64 expansion order of the
plan.
"""
import numpy as np
import pytest

from oracle import direct as DC
from oracle import phs_dense as D
from paper_2608_11462_amd import native as N
from paper_2608_11462_amd import workloads as W
from tests.gpu_util import dev, host, rel

pytestmark = pytest.mark.gpu

ROWS = 4096


def _run(pr, m, nu, precision=N.PHS_FP64):
    k, d = pr.k, (pr.degree if pr.degree >= 0 else D.d_min(pr.k))
    print(f"[case] {pr.name} n={pr.n} k={k} precision={precision}", flush=True)
    pl = N.Plan(dev(pr.xy), k, d)
    c, rho, xi = D.normalize(pr.xy, k)
    assert pl.center == (c[0], c[1]) and pl.scale == rho
    rws = W.sample_rows(11, pr.n, ROWS)
    v = W.rng_for(12).standard_normal(pr.n)
    y = host(pl.matvec(dev(v)))
    e_mv = rel(y[rws], DC.matvec_rows(k, xi, v, rws))
    ym = host(pl.matvec(dev(v), N.PHS_MIXED))
    e_mx = rel(ym[rws], y[rws])
    pl.precond_build(m=m, nu=nu, seed=0)
    w, beta, info = pl.solve(dev(pr.f), rtol=1e-8, precision=precision)
    w, beta = host(w), host(beta)
    Mw = DC.matvec_rows(k, xi, w, rws)
    B = D.poly_block(xi[rws], d)
    res = pr.f[rws] - Mw - B @ beta
    e_res = np.sqrt(np.mean(res ** 2)) / np.sqrt(np.mean(pr.f ** 2))
    tg = pr.targets[:ROWS]
    s = host(pl.eval(dev(w), dev(beta), dev(tg)))
    s_ref = DC.eval_points(k, xi, w, beta, d, (tg - c) * rho)
    e_ev = rel(s, s_ref)
    print(f"{pr.name}: L={pl.leaf_level} order={pl.order} matvec {e_mv:.2e} (mixed vs fp64 "
          f"{e_mx:.2e}) iters={info.iters} (fp32 {info.iters_fp32}, fp64 {info.iters_fp64}, "
          f"fallback {info.fp64_fallback}) outer={info.outer_refinements} "
          f"resid={info.rel_residual:.2e} node-resid {e_res:.2e} eval {e_ev:.2e}")
    assert info.iters == info.iters_fp32 + info.iters_fp64
    assert e_mv <= 1e-10
    assert info.rel_residual <= 1e-8
    assert e_res <= 1e-8
    assert e_ev <= 1e-10
    pl.close()
    return info, w


def test_odd_clustered_full():
    _run(W.odd_clustered(), 50, 1.5)


@pytest.fixture(scope="module")
def large_fp64():
    return _run(W.large_tps(), 30, 1.0)


def test_large_tps_full_fp64(large_fp64):
    info, _ = large_fp64
    assert info.iters <= 40
    assert info.iters_fp32 == 0


def test_large_tps_full_mixed(large_fp64):
    """FP32 far field and near field inside FP64 refinement.  Reaches the same
    gates; the FP32 steps it takes are counted in iters_fp32."""
    info, w = _run(W.large_tps(), 30, 1.0, precision=N.PHS_MIXED)
    assert info.iters_fp32 >= 1


def test_large_tps_full_near32(large_fp64):
    """FP64 far field, FP32 near field: the FP32 steps carry the solve, so the
    weights differ from the FP64 solve's (within the gates)."""
    info, w = _run(W.large_tps(), 30, 1.0, precision=N.PHS_NEAR32)
    assert info.iters_fp32 > 0
    assert not np.array_equal(w, large_fp64[1])
