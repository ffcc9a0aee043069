"""Serving: a stream of solve + evaluate requests of differing n and order,
admitted by slot and device-memory budget while others are on the GPU, with
their PCG iterations sharing launches (continuous batching).

Gates: every request finishes; its weights, coefficients and target values
are bitwise equal to serving it alone through phs_plan + phs_precond_build +
phs_solve + phs_eval with the same options; against the dense FP64 oracle
(eq. phs_linsys_solve, n <= 8000) each served interpolant agrees at its
targets to 1e-8 (max-norm relative) and its node residual
RMS(f - M w - B beta) / RMS(f) is <= 1e-8; the device memory the library holds
while serving (its pool's bytes in use) grows by no more than the budget;
requests really overlapped (more than one active at once) and some waited for
memory.  A request whose plan cannot be built fails with its status on the
build thread while the others are served, and a server closed with builds
still running shuts down cleanly."""
import numpy as np
import pytest

from oracle import phs_dense as D
from paper_2608_11462_amd import native as N
from paper_2608_11462_amd import workloads as W
from tests.gpu_util import dev, host

pytestmark = pytest.mark.gpu


def _requests(seed, count):
    rng = W.rng_for(seed)
    out = []
    for i in range(count):
        n = int(round(np.exp(rng.uniform(np.log(800), np.log(8000)))))
        k = int(rng.choice([2, 3]))
        g = W.rng_for(seed * 100 + i)
        xy = W.clustered_points(g, n) if rng.random() < 0.5 else W.uniform_points(g, n)
        f = W.fourier_field(g, kmax=4)(xy)
        tg = W.uniform_points(g, 300)
        out.append((xy, f, tg, k, int(rng.integers(20, 41))))
    return out


_ORACLE = {}


def _oracle(xy, f, k):
    key = (len(xy), k, float(xy[0, 0]))
    if key not in _ORACLE:
        _ORACLE[key] = D.solve_complement(xy, f, k)
    return _ORACLE[key]


def _alone(xy, f, tg, k, m, precision, rtol):
    pl = N.Plan(dev(xy), k, -1, precision=precision)
    pl.precond_build(m=m, nu=k / 2.0, seed=1)
    w, beta, info = pl.solve(dev(f), rtol=rtol, precision=precision)
    vals = pl.eval(w, beta, dev(tg))
    return host(w), host(beta), host(vals), info


@pytest.mark.parametrize("precision", [N.PHS_FP64, N.PHS_NEAR32])
def test_serving_stream_matches_alone(precision):
    reqs = _requests(77, 10)
    print(f"[case] serving {len(reqs)} requests precision={precision} "
          f"n={[len(r[0]) for r in reqs]}", flush=True)
    # size the budget from the server's own per-request estimate: room for
    # about three of the largest requests, so later ones wait for memory
    probe = N.Server(hbm_budget=1 << 40)
    est = [probe.poll(probe.submit(dev(r[0]), dev(r[1]), r[3], targets=dev(r[2]), m=r[4],
                                   nu=r[3] / 2.0, seed=1)).bytes for r in reqs]
    probe.close()
    budget = 3 * max(est)
    in_use0 = N.memory_stats()[2]
    srv = N.Server(hbm_budget=budget, max_active=6, precision=precision, rtol=1e-9)
    ids = []
    pending = list(range(len(reqs)))
    max_active, waited, steps = 0, False, 0
    while True:
        # arrivals: two new requests every third step
        if pending and steps % 3 == 0:
            for _ in range(2):
                if pending:
                    i = pending.pop(0)
                    xy, f, tg, k, m = reqs[i]
                    ids.append(srv.submit(dev(xy), dev(f), k, targets=dev(tg), m=m,
                                          nu=k / 2.0, seed=1))
        active, queued = srv.step()
        steps += 1
        max_active = max(max_active, active)
        used, peak = srv.memory()
        if queued and active:
            waited = True
        assert used <= budget and peak <= budget
        held = N.memory_stats()[2] - in_use0  # device bytes the library really holds
        assert held <= budget, (held, budget)
        if not pending and active == 0 and queued == 0:
            break
        assert steps < 20000
    print(f"steps={steps} max_active={max_active} waited={waited} peak={peak} budget={budget}")
    assert max_active >= 2
    for rid, (xy, f, tg, k, m) in zip(ids, reqs):
        inf = srv.poll(rid)
        assert inf.state == N.PHS_REQ_DONE and inf.status == 0, (rid, inf.state, inf.status)
        w, beta, vals = (host(t) for t in srv.result(rid))
        wa, ba, va, ia = _alone(xy, f, tg, k, m, precision, 1e-9)
        print(f"req {rid} n={len(xy)} k={k} iters {inf.iters}/{ia.iters} "
              f"resid {inf.rel_residual:.2e} latency {inf.t_done - inf.t_submit:.4f}s "
              f"wait {inf.t_admit - inf.t_submit:.4f}s")
        assert inf.iters == ia.iters
        np.testing.assert_array_equal(w, wa)
        np.testing.assert_array_equal(beta, ba)
        np.testing.assert_array_equal(vals, va)
        # against the dense oracle
        ref = _oracle(xy, f, k)
        s_ref = D.interpolant(ref, k, tg)
        e_s = np.abs(vals - s_ref).max() / np.abs(s_ref).max()
        xi = ref["xi"]
        res = f - D.kernel_matrix(k, xi, xi) @ w - D.poly_block(xi, ref["degree"]) @ beta
        e_r = np.sqrt(np.mean(res ** 2)) / np.sqrt(np.mean(f ** 2))
        print(f"    vs oracle: interpolant {e_s:.2e} node residual {e_r:.2e}")
        assert e_s <= 1e-8
        assert e_r <= 1e-8
    srv.close()


def test_oversized_request_fails_cleanly():
    xy = W.uniform_points(W.rng_for(5), 3000)
    f = W.f_small(xy)
    srv = N.Server(hbm_budget=1 << 20)  # 1 MiB: too small for any request
    rid = srv.submit(dev(xy), dev(f), 2, targets=dev(xy[:10]))
    srv.step()
    inf = srv.poll(rid)
    assert inf.state == N.PHS_REQ_FAILED and inf.status == 6  # PHS_ERR_OUT_OF_MEMORY
    assert srv.memory() == (0, 0)
    srv.close()


def test_failed_build_and_close_during_builds():
    """A request whose plan cannot be built (two coincident nodes) fails on the
    build thread with its status while the others are served; a server closed
    while builds are in flight shuts down cleanly."""
    print("[case] serving: failing build among good requests", flush=True)
    reqs = _requests(91, 4)
    bad_xy = reqs[1][0].copy()
    bad_xy[7] = bad_xy[3]  # duplicate node
    srv = N.Server(hbm_budget=1 << 34, max_active=8)
    ids = []
    for i, (xy, f, tg, k, m) in enumerate(reqs):
        ids.append(srv.submit(dev(bad_xy if i == 1 else xy), dev(f), k, targets=dev(tg), m=m,
                              nu=k / 2.0, seed=1))
    steps = 0
    while True:
        active, queued = srv.step()
        steps += 1
        if active == 0 and queued == 0:
            break
        assert steps < 20000
    for i, rid in enumerate(ids):
        inf = srv.poll(rid)
        if i == 1:
            assert inf.state == N.PHS_REQ_FAILED and inf.status == 2  # DUPLICATE_POINTS
        else:
            assert inf.state == N.PHS_REQ_DONE and inf.status == 0, (i, inf.state, inf.status)
            xy, f, tg, k, m = reqs[i]
            wa, ba, va, _ = _alone(xy, f, tg, k, m, N.PHS_FP64, 1e-8)
            w, beta, vals = (host(t) for t in srv.result(rid))
            np.testing.assert_array_equal(vals, va)
    assert srv.memory()[0] == 0
    srv.close()
    # close with builds still running
    srv = N.Server(hbm_budget=1 << 34, max_active=8)
    for xy, f, tg, k, m in reqs:
        srv.submit(dev(xy), dev(f), k, targets=dev(tg), m=m, nu=k / 2.0, seed=1)
    srv.step()
    srv.close()
