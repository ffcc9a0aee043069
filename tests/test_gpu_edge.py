"""Edge cases and error paths through the C ABI."""
import numpy as np
import pytest

from oracle import phs_dense as D
from paper_2608_11462_amd import native as N
from paper_2608_11462_amd import workloads as W
from tests.gpu_util import dev, host, rel

pytestmark = pytest.mark.gpu


def test_duplicate_nodes_rejected():
    xy = W.uniform_points(W.rng_for(1), 500)
    xy[17] = xy[301]
    with pytest.raises(N.PHSError) as ei:
        N.Plan(dev(xy), 2)
    assert ei.value.name == "PHS_ERR_DUPLICATE_POINTS"


def test_collinear_nodes_unisolvent():
    t = np.linspace(0.0, 1.0, 200)
    xy = np.stack([t, 0.5 * t + 0.1], axis=1)
    with pytest.raises(N.PHSError) as ei:
        N.Plan(dev(xy), 2)
    assert ei.value.name == "PHS_ERR_UNISOLVENT"


def test_bad_arguments():
    xy = W.uniform_points(W.rng_for(2), 100)
    for kw in (dict(k=0), dict(k=5), dict(k=2, degree=0), dict(k=4, degree=1)):
        with pytest.raises(N.PHSError) as ei:
            N.Plan(dev(xy), kw["k"], kw.get("degree", -1))
        assert ei.value.name == "PHS_ERR_INVALID_ARGUMENT"
    pl = N.Plan(dev(xy), 2)
    with pytest.raises(N.PHSError):
        pl.precond_build(m=200)
    with pytest.raises(N.PHSError):
        pl.precond_build(nu=0.75)


def test_minimal_node_set():
    """n = S: the polynomial interpolates alone and w = 0."""
    xy = W.uniform_points(W.rng_for(3), 3)
    f = W.f_small(xy)
    pl = N.Plan(dev(xy), 2, 1)
    w, beta, info = pl.solve(dev(f))
    ref = D.solve_complement(xy, f, 2, 1)
    assert np.all(host(w) == 0.0)
    np.testing.assert_allclose(host(beta), ref["beta"], rtol=1e-10, atol=1e-12)


def test_polynomial_data_gives_zero_weights():
    xy = W.uniform_points(W.rng_for(4), 1500)
    f = 1.0 + 2.0 * xy[:, 0] - 3.0 * xy[:, 1]
    pl = N.Plan(dev(xy), 2, 1)
    pl.precond_build(seed=1)
    w, beta, info = pl.solve(dev(f))
    assert info.iters == 0
    assert np.all(host(w) == 0.0)
    tg = W.uniform_points(W.rng_for(5), 50)
    s = host(pl.eval(w, beta, dev(tg)))
    np.testing.assert_allclose(s, 1.0 + 2.0 * tg[:, 0] - 3.0 * tg[:, 1], rtol=1e-11, atol=1e-11)


def test_targets_on_nodes_and_outside():
    pr = W.small_tps(n=1200)
    ref = D.solve_complement(pr.xy, pr.f, 2, 1)
    pl = N.Plan(dev(pr.xy), 2, 1)
    tg = np.concatenate([pr.xy[:40], W.uniform_points(W.rng_for(6), 40) * 4.0 - 1.5])
    s = host(pl.eval(dev(ref["w"]), dev(ref["beta"]), dev(tg)))
    s_ref = D.interpolant(ref, 2, tg)
    assert np.abs(s - s_ref).max() <= 1e-10 * np.abs(s_ref).max()
    # interpolation at the nodes
    assert np.abs(s[:40] - pr.f[:40]).max() <= 1e-8 * np.abs(pr.f).max()


def test_empty_eval_and_maxit():
    pr = W.small_tps(n=800)
    pl = N.Plan(dev(pr.xy), 2, 1)
    out = pl.eval(dev(np.zeros(pr.n)), dev(np.zeros(3)), dev(np.zeros((0, 2))))
    assert out.numel() == 0
    w, beta, info = pl.solve(dev(pr.f), maxit=2, raise_on_error=False)
    assert info.status == "PHS_ERR_NOT_CONVERGED" and info.iters == 2
