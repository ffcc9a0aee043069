"""The C-ABI contract on ownership and preconditioner state.

* phs_matvec (every precision), phs_solve (every precision), phs_eval and
  phs_batch_solve allocate no device memory: the library pool's allocation
  counter (phs_memory_stats) is the same before and after them, including on
  their first call after phs_plan / phs_batch_create.
* A preconditioner rebuild that fails leaves the plan's previous factor in
  place (the next solve is bitwise the earlier one); a rebuild that succeeds
  is picked up by the next solve (bitwise equal to a fresh plan built with the
  same options)."""
import numpy as np
import pytest

from paper_2608_11462_amd import native as N
from paper_2608_11462_amd import workloads as W
from tests.gpu_util import dev, host

pytestmark = pytest.mark.gpu


def _allocs():
    return N.memory_stats()[0]


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_calls_allocate_nothing(k):
    rng = W.rng_for(600 + k)
    xy = W.clustered_points(rng, 6000)
    f = W.fourier_field(rng, kmax=4)(xy)
    tg = W.uniform_points(rng, 500) * 1.4 - 0.2
    print(f"[case] no-allocation k={k}", flush=True)
    pl = N.Plan(dev(xy), k)
    v = dev(rng.standard_normal(len(xy)))
    a0 = _allocs()
    for prec in (N.PHS_FP64, N.PHS_MIXED, N.PHS_NEAR32):
        pl.matvec(v, prec)
    w, beta, _ = pl.solve(dev(f), rtol=1e-6, maxit=40, raise_on_error=False)  # identity
    assert _allocs() == a0
    pl.precond_build(m=20, nu=k / 2.0, seed=2)
    a1 = _allocs()
    for prec in (N.PHS_FP64, N.PHS_MIXED, N.PHS_NEAR32):
        w, beta, info = pl.solve(dev(f), rtol=1e-8, precision=prec)
        assert info.status == "PHS_OK"
    vals = pl.eval(w, beta, dev(tg))
    F2 = dev(np.stack([f, np.cos(3 * xy[:, 0])], 1))
    pl.matvec(F2)
    pl.solve(F2, rtol=1e-8)
    host(vals)
    assert _allocs() == a1
    pl.close()


def test_batch_solve_allocates_nothing():
    print("[case] batch no-allocation", flush=True)
    plans, fs = [], []
    for i, k in enumerate((1, 2, 3, 4)):
        rng = W.rng_for(620 + i)
        xy = W.uniform_points(rng, 1500 + 700 * i)
        plans.append(N.Plan(dev(xy), k))
        plans[-1].precond_build(m=24, nu=k / 2.0, seed=i)
        fs.append(dev(W.fourier_field(rng, kmax=4)(xy)))
    b = N.Batch(plans)
    a0 = _allocs()
    for prec in (N.PHS_FP64, N.PHS_MIXED):
        out, infos = b.solve(fs, rtol=1e-8, precision=prec)
        assert all(i.status == "PHS_OK" for i in infos)
    host(out[0][0])
    assert _allocs() == a0
    b.close()
    for p in plans:
        p.close()


def test_precond_rebuild_keeps_or_replaces_factor():
    pr = W.small_tps(n=3000)
    print("[case] precond rebuild", flush=True)
    pl = N.Plan(dev(pr.xy), 2, 1)
    pl.precond_build(m=30, nu=1.0, seed=4)
    w1, b1, _ = pl.solve(dev(pr.f), rtol=1e-9)
    w1 = host(w1)
    # an invalid rebuild fails and leaves the factor in place
    with pytest.raises(N.PHSError):
        pl.precond_build(m=30, nu=0.7, seed=9)
    w2, _, _ = pl.solve(dev(pr.f), rtol=1e-9)
    np.testing.assert_array_equal(host(w2), w1)
    # a valid rebuild with another seed replaces it
    pl.precond_build(m=30, nu=1.0, seed=9)
    w3, _, _ = pl.solve(dev(pr.f), rtol=1e-9)
    fresh = N.Plan(dev(pr.xy), 2, 1)
    fresh.precond_build(m=30, nu=1.0, seed=9)
    w4, _, _ = fresh.solve(dev(pr.f), rtol=1e-9)
    w3, w4 = host(w3), host(w4)
    np.testing.assert_array_equal(w3, w4)
    assert not np.array_equal(w3, w1)
    pl.close()
    fresh.close()
