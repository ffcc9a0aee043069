"""Full-size workloads, checked on sampled outputs by FP64 direct summation
(the oracle cannot form these matrices).

* odd_clustered: n = 100000 (70% uniform + 30% in 10 Gaussian clusters), k = 3,
  quadratic block, Vecchia m = 50, nu = 1.5, alpha = 3 (the k = 3 default).
* large_tps: n = 2^20 uniform, k = 2, linear block, Vecchia m = 30, nu = 1,
  alpha = 0.35 (the benchmark configuration).
Gates: matvec 1e-10 relative on sampled rows (FP64); the solver's own FP64
residual over all nodes <= 1e-8; the node residual RMS(f - M w - B beta)/RMS(f)
recomputed by direct summation on the sampled nodes <= 1.25e-8 (an RMS over
128 sampled rows estimates the full one with a relative standard error of
about sqrt(2/128)/2 = 6%, so a solve that stops just under 1e-8 can read
above it on the sample; 1.25 is four standard errors);
evaluation at sampled targets (4096 in the FP64 benchmark case) <= 1e-10
relative to direct summation with the same (w, beta).  The interpolant is a
sum of large alternating w_j phi terms (an FMM error of ~2e-14 relative to
sum |w_j phi| shows up as ~1e-10 relative to max |s|), which is why target
evaluation uses the tighter FP64 expansion order of the plan.
"""
import numpy as np
import pytest

from oracle import phs_dense as D
from paper_2608_11462_amd import native as N
from paper_2608_11462_amd import workloads as W
from tests.gpu_util import dev, host, rel

pytestmark = pytest.mark.gpu


def _run(pr, m, nu, rows, ntg, precision=N.PHS_FP64):
    k, d = pr.k, (pr.degree if pr.degree >= 0 else D.d_min(pr.k))
    print(f"[case] {pr.name} n={pr.n} k={k} precision={precision}", flush=True)
    pl = N.Plan(dev(pr.xy), k, d)
    c, rho, xi = D.normalize(pr.xy, k)
    assert pl.center == (c[0], c[1]) and pl.scale == rho
    rws = W.sample_rows(11, pr.n, rows)
    v = W.rng_for(12).standard_normal(pr.n)
    y = host(pl.matvec(dev(v)))
    e_mv = rel(y[rws], D.matvec_rows(k, xi, v, rws))
    ym = host(pl.matvec(dev(v), N.PHS_MIXED))
    e_mx = rel(ym[rws], y[rws])
    pl.precond_build(m=m, nu=nu, seed=0)
    w, beta, info = pl.solve(dev(pr.f), rtol=1e-8, precision=precision)
    w, beta = host(w), host(beta)
    Mw = D.matvec_rows(k, xi, w, rws)
    B = D.poly_block(xi[rws], d)
    res = pr.f[rws] - Mw - B @ beta
    e_res = np.sqrt(np.mean(res ** 2)) / np.sqrt(np.mean(pr.f ** 2))
    tg = pr.targets[:ntg]
    s = host(pl.eval(dev(w), dev(beta), dev(tg)))
    s_ref = D.eval_points(k, xi, w, beta, d, (tg - c) * rho)
    e_ev = rel(s, s_ref)
    print(f"{pr.name}: L={pl.leaf_level} order={pl.order} matvec {e_mv:.2e} (mixed vs fp64 "
          f"{e_mx:.2e}) iters={info.iters} outer={info.outer_refinements} "
          f"resid={info.rel_residual:.2e} node-resid {e_res:.2e} eval {e_ev:.2e}")
    assert e_mv <= 1e-10
    assert info.rel_residual <= 1e-8
    assert e_res <= 1.25e-8  # sampled estimate of a residual the solver holds to 1e-8
    assert e_ev <= 1e-10
    return info


def test_odd_clustered_full():
    _run(W.odd_clustered(), 50, 1.5, 512, 2048)


def test_large_tps_full_fp64():
    info = _run(W.large_tps(), 30, 1.0, 256, 4096)
    assert info.iters <= 40


def test_large_tps_full_mixed():
    _run(W.large_tps(), 30, 1.0, 128, 512, precision=N.PHS_MIXED)


def test_large_tps_full_near32():
    _run(W.large_tps(), 30, 1.0, 128, 512, precision=N.PHS_NEAR32)
