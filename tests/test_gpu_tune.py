"""The tuners on the GPU path.

* phs_tune_precond: the preconditioner it leaves on the plan gives a solve
  that matches the dense oracle (interpolant <= 1e-8, weights within the
  floor-aware gate), and its measured build + solve time is no worse than
  the library defaults' on the same problem (the defaults are one of its
  trials).
* phs_autotune_plan: the plan options it returns give a matvec within the
  requested tolerance of the oracle's own direct sums on 4096 sampled rows
  (independent of the exact GPU sum the autotuner measured against)."""
import numpy as np
import pytest

from oracle import direct as DC
from oracle import phs_dense as D
from paper_2608_11462_amd import native as N
from paper_2608_11462_amd import workloads as W
from tests.gpu_util import dev, host, rel

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("k", [2, 3])
def test_tune_precond_leaves_a_correct_preconditioner(k):
    rng = W.rng_for(900 + k)
    xy = W.clustered_points(rng, 3000) if k == 3 else W.uniform_points(rng, 3000)
    f = W.fourier_field(rng, kmax=4)(xy)
    print(f"[case] tune_precond k={k}", flush=True)
    pl = N.Plan(dev(xy), k)
    r = pl.tune_precond(dev(f), rtol=1e-10, max_evals=10)
    print(f"k={k}: best m={r['m']} nu={r['nu']} alpha={r['alpha']:.3g} "
          f"{r['seconds'] * 1e3:.2f} ms / {r['iters']} it (defaults "
          f"{r['default_seconds'] * 1e3:.2f} ms / {r['default_iters']} it), {r['evals']} trials")
    assert r["seconds"] <= r["default_seconds"]
    assert r["rel_residual"] <= 1e-10
    w, beta, info = pl.solve(dev(f), rtol=1e-10)
    ref = D.solve_complement(xy, f, k)
    bk = D.solve_bunch_kaufman(xy, f, k)
    tg = W.uniform_points(rng, 200)
    s = host(pl.eval(w, beta, dev(tg)))
    s_ref = D.interpolant(ref, k, tg)
    assert np.abs(s - s_ref).max() / np.abs(s_ref).max() <= 1e-8
    assert rel(host(w), ref["w"]) <= max(1e-8, 10 * rel(bk["w"], ref["w"]))
    pl.close()


@pytest.mark.parametrize("k,n,tol", [(2, 3000, 1e-12), (2, 60000, 1e-10), (3, 60000, 1e-11),
                                     (4, 30000, 1e-10)])
def test_autotune_plan_meets_its_tolerance(k, n, tol):
    rng = W.rng_for(910 + k + n)
    xy = W.clustered_points(rng, n) if k % 2 else W.uniform_points(rng, n)
    print(f"[case] autotune k={k} n={n} tol={tol}", flush=True)
    kw, rep = N.autotune_plan(dev(xy), k, matvec_tol=tol)
    print(f"k={k} n={n}: chose {kw} ({rep})")
    assert rep["rel_error"] <= tol
    pl = N.Plan(dev(xy), k, **kw)
    c, rho, xi = D.normalize(xy, k)
    v = W.rng_for(911).standard_normal(n)
    rows = W.sample_rows(912, n, 4096)
    e = rel(host(pl.matvec(dev(v)))[rows], DC.matvec_rows(k, xi, v, rows))
    print(f"  oracle-checked matvec error {e:.2e}")
    assert e <= tol
    pl.close()
