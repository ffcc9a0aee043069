"""Benchmark: one MI355X, n = 2^20 thin-plate-spline interpolation.

A step is one pass of the whole hot path on the resident synthetic workload:
plan (normalise, quadtree, polynomial block + QR) -> Vecchia/Matern
preconditioner build -> projected PCG to 1e-8 relative residual (FMM matvecs)
-> beta recovery -> evaluation at 10^4 targets.  Inputs live in HBM before the
timed region starts.

    python bench.py [--steps K] [--warmup W] [--precision fp64|mixed]

Prints ONE JSON line.  `value` is solved nodes per second (Mpts/s) over the
whole step; the line also carries the solve seconds, PCG iterations, the FMM
matvec throughput in FP64 and mixed precision, the roofline of the dominant
kernel (timed with HIP events on its own stream inside the timed region) and
the CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time
from pathlib import Path

import numpy as np

ROOT = Path(__file__).resolve().parent
sys.path.insert(0, str(ROOT))

FP64_PEAK_TFLOPS = 78.6   # MI355X vector FP64 (and FP64 matrix)
FP32_PEAK_TFLOPS = 157.3  # MI355X vector FP32 with packed math
FP32_NOPACK_TFLOPS = 78.6  # MI355X vector FP32 without packed math (the kernels are built without it)

# Algorithmic flop counts used for the rooflines (one convention throughout):
#  near-field pair: 2 sub, r^2 (mul + fma = 3), 1 transcendental counted as 1,
#  accumulate (fma = 2), one scale -> 9 flops
#  local-expansion evaluation per node and density: P complex multiply-adds,
#  8 flops each -> 8 P
#  M2L per (target, source, density): (P+1)^2 real-by-complex MACs (4 flops)
#  + 12 (P+1) for the two diagonal scalings
FLOP_PAIR = 9
N_P2P = 1 << 16  # nodes of the all-pairs P2P measurement


def progress(msg: str) -> None:
    """One line on stderr as a leg finishes a piece of work (the JSON result
    stays the only line on stdout)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", choices=["fp64", "mixed", "near32"], default="fp64")
    ap.add_argument("--no-precision-leg", action="store_true",
                    help="skip timing the solve in the two reduced-precision forms")
    ap.add_argument("--n", type=int, default=1 << 20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true")
    # one elementwise kernel reading 1 GiB and writing 1 GiB before the steps:
    # the reference for scaling rocprofv3 FETCH_SIZE / WRITE_SIZE counters
    ap.add_argument("--copy-calibration", action="store_true")
    # serving (Poisson stream) and batched (many problems, 4 right-hand sides) legs
    ap.add_argument("--serve-requests", type=int, default=64)
    ap.add_argument("--batch-problems", type=int, default=256)
    # 512-request Poisson streams at 0.8, 1.0 and 1.2 x the load the plain
    # FP64 path sustains alone (several minutes; off by default)
    ap.add_argument("--serve-sweep", action="store_true")
    # retune (phs_tune_precond) and re-solve the batched problems that miss 1e-8
    ap.add_argument("--retune", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-crossover", action="store_true")
    ap.add_argument("--no-tree-leg", action="store_true",
                    help="skip the uniform-against-clustered tree cost leg")
    return ap.parse_args()


def tree_work(order_leaf: np.ndarray, L: int, n: int):
    """Near-field pair count and leaf counts from the plan's leaf keys."""
    G = 1 << L
    counts = np.bincount(order_leaf, minlength=G * G).reshape(G, G)  # [iy, ix]
    pad = np.pad(counts, 1)
    nb = sum(pad[1 + dy:1 + dy + G, 1 + dx:1 + dx + G]
             for dy in (-1, 0, 1) for dx in (-1, 0, 1))
    pairs = int((counts * nb).sum())
    # interaction-list pairs per level (uniform tree, boundary clipped)
    m2l_pairs = 0
    for l in range(2, L + 1):
        g = 1 << l
        ii = np.arange(g)
        cnt = 0
        for oy in range(-3, 4):
            for ox in range(-3, 4):
                if abs(ox) <= 1 and abs(oy) <= 1:
                    continue
                jx = ii + ox
                okx = (jx >= 0) & (jx < g) & (np.abs((jx >> 1) - (ii >> 1)) <= 1)
                jy = ii + oy
                oky = (jy >= 0) & (jy < g) & (np.abs((jy >> 1) - (ii >> 1)) <= 1)
                cnt += int(okx.sum()) * int(oky.sum())
        m2l_pairs += cnt
    return pairs, m2l_pairs


def source_sha(name: str) -> str:
    """Hash of the source file that holds a kernel (counters taken on another
    version of that file are not reported)."""
    h = hashlib.sha256()
    h.update((ROOT / "paper_2608_11462_amd" / "csrc" / name).read_bytes())
    return h.hexdigest()[:16]


def stored_traffic(kernel: str, workload: str):
    """HBM bytes per launch from committed rocprofv3 counter runs, if they were
    taken on the current source of the kernel."""
    f = ROOT / "profiles" / f"traffic_{kernel}_{workload}.json"
    if not f.exists():
        return None
    d = json.loads(f.read_text())
    if d.get("source_sha") != source_sha(d["source"]):
        return None
    return d.get("bytes_per_launch")


def cpu_baseline(checks=None, seed: int = 3, n_s: int = 6144, n_t: int = 10000):
    """The CPU oracle timed on this host, on bounded samples of the workloads:
    (1) dense FP64 complement solve + 10^4-target evaluation on n_s nodes of
    the n = 2^20 workload's distribution (median of 3; this is `value`), and a
    scaling sweep of the same dense solve at n = 2k..16k (one run each, O(n^3));
    (2) the direct-summation matvec of the n = 1e5 odd-order workload, timed on
    4096 rows and stated as points per second of a full matvec; (3) the
    4096-row sampled checker of the n = 2^20 workload.  `checks`: weights and
    coefficients of the benchmark's solves, whose node residual
    RMS(f - M w - B beta) / RMS(f) the oracle recomputes on 4096 sampled nodes."""
    from oracle import direct as DC
    from oracle import phs_dense as D
    from paper_2608_11462_amd import workloads as W
    try:
        from threadpoolctl import threadpool_info
        blas = max((i.get("num_threads", 0) for i in threadpool_info()
                    if i.get("user_api") == "blas"), default=None)
    except Exception:  # threadpoolctl missing: report unknown
        blas = None
    pr = W.large_tps(seed=seed, n=n_s, n_targets=n_t)
    ts = []
    for _ in range(3):
        t0 = time.perf_counter()
        sol = D.solve_complement(pr.xy, pr.f, 2, 1)
        D.interpolant(sol, 2, pr.targets)
        ts.append(time.perf_counter() - t0)
    t = float(np.median(ts))
    sweep = {}
    for ns in (2000, 4000, 8000, 16000):
        p2 = W.small_tps(n=ns, n_targets=500)
        t0 = time.perf_counter()
        sol = D.solve_complement(p2.xy, p2.f, 2, 1)
        D.interpolant(sol, 2, p2.targets)
        sweep[str(ns)] = round(time.perf_counter() - t0, 3)
        progress(f"CPU oracle: dense solve n={ns} in {sweep[str(ns)]} s")
    oc = W.odd_clustered()
    _, _, xi_c = D.normalize(oc.xy, 3)
    rows = W.sample_rows(11, oc.n, 4096)
    vv = W.rng_for(12).standard_normal(oc.n)
    t0 = time.perf_counter()
    DC.matvec_rows(3, xi_c, vv, rows)
    t_rows = time.perf_counter() - t0
    lt = W.large_tps()
    _, _, xi_l = D.normalize(lt.xy, 2)
    rows_l = W.sample_rows(11, lt.n, 4096)
    t0 = time.perf_counter()
    DC.matvec_rows(2, xi_l, W.rng_for(12).standard_normal(lt.n), rows_l)
    t_check = time.perf_counter() - t0
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count()
    out = {"value": n_s / t / 1e6, "unit": "Mpts/s", "cores": cores, "kind": "oracle",
           "blas_threads": blas, "c_threads": DC.threads(),
           "sample": f"dense FP64 complement solve + {n_t}-target evaluation on {n_s} nodes "
                     f"of the same workload (median of 3: {t:.2f} s)",
           "dense_solve_sweep_s": sweep,
           "direct_matvec_odd_clustered_pts_per_s": round(oc.n / (t_rows * oc.n / 4096), 1),
           "direct_matvec_note": "C direct summation of 4096 rows of the n = 1e5 k = 3 "
                                 f"matvec in {t_rows:.2f} s, scaled to a full matvec",
           "checker_4096_rows_large_tps_s": round(t_check, 3)}
    if checks:
        xy_l = lt.xy
        res = {}
        for name, (w, beta) in checks.items():
            Mw = DC.matvec_rows(2, xi_l, w, rows_l)
            r = lt.f[rows_l] - Mw - D.poly_block(xi_l[rows_l], 1) @ beta
            res[name] = float(np.sqrt(np.mean(r ** 2)) / np.sqrt(np.mean(lt.f ** 2)))
        out["node_residual_vs_oracle_4096"] = res
    return out


def crossover_leg(N, W, torch):
    """FMM against the exact (all-pairs) matvec on plans of the small
    thin-plate workload (uniform nodes, k = 2): FP64 matvec milliseconds per
    size, and the smallest size where the FMM is faster."""
    dev = torch.device("cuda")
    rows = []
    cross = None
    for n in (1000, 2000, 4000, 8000, 16000, 32000, 64000, 128000):
        pr = W.small_tps(n=n, n_targets=10)
        xy = torch.as_tensor(pr.xy, device=dev)
        v = torch.as_tensor(W.rng_for(5).standard_normal(n), device=dev)
        t = {}
        for name, kind in (("fmm", N.PHS_MATVEC_FMM), ("direct", N.PHS_MATVEC_DIRECT)):
            pl = N.Plan(xy, 2, 1, matvec=kind)
            for _ in range(3):
                pl.matvec(v)
            torch.cuda.synchronize()
            reps = 20
            t0 = time.perf_counter()
            for _ in range(reps):
                pl.matvec(v)
            torch.cuda.synchronize()
            t[name] = (time.perf_counter() - t0) / reps * 1e3
            pl.close()
        rows.append({"n": n, "fmm_ms": round(t["fmm"], 4), "direct_ms": round(t["direct"], 4)})
        if cross is None and t["fmm"] < t["direct"]:
            cross = n
    return {"k": 2, "matvec_ms": rows, "fmm_faster_from_n": cross}


def tree_leg(N, W, torch, n: int = 1 << 20):
    """Cost of the uniform quadtree on clustered nodes: the FP64 k = 2 matvec
    on n uniform nodes against n nodes of which 30 % lie in ten Gaussian
    clusters of sigma 0.02 (the serving stream's clustered requests).  The
    clustered tree is deeper (its leaf level keeps the largest leaf below a
    bound), so empty boxes pay M2L and sparse leaves pay the near-field pass;
    the uniform matvec at the same n is what an adaptive tree could at best
    recover.  Leaf and M2L milliseconds from HIP events, the whole matvec by
    wall clock."""
    dev = torch.device("cuda")
    out = {"n": n, "k": 2}
    for name, xy in (("uniform", W.uniform_points(W.rng_for(31), n)),
                     ("clustered", W.clustered_points(W.rng_for(32), n))):
        pl = N.Plan(torch.as_tensor(xy, device=dev), 2, 1)
        v = torch.as_tensor(W.rng_for(33).standard_normal(n), device=dev)
        for _ in range(3):
            pl.matvec(v)
        torch.cuda.synchronize()
        reps = 10
        t0 = time.perf_counter()
        for _ in range(reps):
            pl.matvec(v)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / reps * 1e3
        N.profile_enable(2)
        N.profile_read()
        for _ in range(reps):
            pl.matvec(v)
        torch.cuda.synchronize()
        prof = N.profile_read()
        N.profile_enable(False)
        out[name] = {"leaf_level": pl.leaf_level, "matvec_ms": round(wall, 4),
                     **{k + "_ms": round(prof[k][1] / prof[k][0], 4)
                        for k in ("leaf_eval", "m2l") if k in prof}}
        pl.close()
    out["clustered_over_uniform"] = round(out["clustered"]["matvec_ms"]
                                          / out["uniform"]["matvec_ms"], 3)
    # the clustered nodes at other leaf sizes (the level follows from the
    # size, deepened while the largest leaf exceeds 16 times it)
    xy = torch.as_tensor(W.clustered_points(W.rng_for(32), n), device=dev)
    v = torch.as_tensor(W.rng_for(33).standard_normal(n), device=dev)
    rows = []
    for ls in (256, 64, 16):
        pl = N.Plan(xy, 2, 1, leaf_size=ls)
        for _ in range(3):
            pl.matvec(v)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(10):
            pl.matvec(v)
        torch.cuda.synchronize()
        rows.append({"leaf_size": ls, "leaf_level": pl.leaf_level,
                     "matvec_ms": round((time.perf_counter() - t0) / 10 * 1e3, 4)})
        pl.close()
    out["clustered_by_leaf_size"] = rows
    return out


def serve_leg(N, W, torch, n_req: int, loads=(0.8,)):
    """Poisson stream of solve + evaluate requests (n log-uniform in [1e3, 1e6],
    k in {2, 3}, 10^4 targets) through the server at 80% of the load the plain
    FP64 path sustains serving each request alone; FIFO serve-alone latencies
    follow from the measured alone service times and the same arrivals."""
    reqs = W.stream(n_requests=n_req, rate=1.0)
    dev = torch.device("cuda")
    items = [(torch.as_tensor(r.problem.xy, device=dev), torch.as_tensor(r.problem.f, device=dev),
              torch.as_tensor(r.problem.targets, device=dev), r.problem.k,
              r.problem.precond["m"]) for r in reqs]
    torch.cuda.synchronize()

    def alone(it):
        xy, f, tg, k, m = it
        pl = N.Plan(xy, k, -1)
        pl.precond_build(m=m, nu=k / 2.0, seed=0)
        w, b, info = pl.solve(f, rtol=1e-8)
        pl.eval(w, b, tg)
        torch.cuda.synchronize()
        pl.close()
        return info.rel_residual

    alone(items[0])  # warm-up
    t_alone = []
    for i, it in enumerate(items):
        t0 = time.perf_counter()
        alone(it)
        t_alone.append(time.perf_counter() - t0)
        if (i + 1) % 64 == 0:
            progress(f"serving: {i + 1} requests timed alone")
    results = []
    for load in loads:
        results.append(_serve_at(N, items, reqs, t_alone, load, n_req))
        progress(f"serving: load {load} done")
    return results[0] if len(results) == 1 else {"loads": results}


def _serve_at(N, items, reqs, t_alone, load, n_req):
    lam = load / float(np.mean(t_alone))
    arr = [r.t_arrival / lam for r in reqs]
    fin, lat_alone = 0.0, []
    for a, ts in zip(arr, t_alone):
        fin = max(fin, a) + ts
        lat_alone.append(fin - a)
    srv = N.Server(max_active=64, precision=N.PHS_FP64, rtol=1e-8)
    ids, sub = [], []
    t0 = time.perf_counter()
    nxt = 0
    while True:
        now = time.perf_counter() - t0
        while nxt < len(items) and arr[nxt] <= now:
            xy, f, tg, k, m = items[nxt]
            ids.append(srv.submit(xy, f, k, targets=tg, m=m, nu=k / 2.0, seed=0))
            sub.append(time.perf_counter() - t0)
            nxt += 1
        active, queued = srv.step()
        if nxt % 64 == 0 and nxt and nxt != getattr(srv, "_reported", -1):
            srv._reported = nxt
            progress(f"serving: {nxt} requests submitted")
        if active == 0 and queued == 0:
            if nxt == len(items):
                break
            time.sleep(max(0.0, arr[nxt] - (time.perf_counter() - t0)))
    makespan = time.perf_counter() - t0 - arr[0]
    lat, worst = [], 0.0
    for i, rid in enumerate(ids):
        inf = srv.poll(rid)
        if inf.state != N.PHS_REQ_DONE or inf.status != 0:
            raise RuntimeError(f"serving request {rid} failed (state {inf.state}, "
                               f"status {inf.status})")
        lat.append((inf.t_done - inf.t_submit) + (sub[i] - arr[i]))
        worst = max(worst, inf.rel_residual)
    _, peak = srv.memory()
    srv.close()
    q = lambda v, p: round(1e3 * float(np.percentile(v, p)), 3)
    return {"requests": n_req, "load": load, "rate_per_s": round(lam, 3),
            "p50_ms": q(lat, 50), "p99_ms": q(lat, 99),
            "solves_per_s": round(n_req / makespan, 3),
            "alone_fifo_p50_ms": q(lat_alone, 50), "alone_fifo_p99_ms": q(lat_alone, 99),
            "alone_solves_per_s": round(n_req / (fin - arr[0]), 3),
            "mean_alone_ms": round(1e3 * float(np.mean(t_alone)), 3),
            "worst_rel_residual": worst, "peak_hbm_bytes": peak}


def _info_fields(info):
    return {"pcg_iters": info.iters, "iters_fp32": info.iters_fp32,
            "iters_fp64": info.iters_fp64, "fp64_fallback": info.fp64_fallback,
            "outer_refinements": info.outer_refinements, "rel_residual_fp64": info.rel_residual}


def precision_leg(N, torch, xy, f, tg, steps: int = 2):
    """The same n = 2^20 solve (plan + preconditioner + solve to 1e-8 + evaluation)
    in the two reduced-precision forms, beside the FP64 step: FP32 FMM with FP64
    Krylov and FP64 residual refinement, and FP64 far field with an FP32 near
    field.  All reach the FP64 residual 1e-8.  Returns the timings and the
    weights of each form (checked against the oracle in the CPU leg)."""
    out, sols = {}, {}
    for name, prec in (("mixed", N.PHS_MIXED), ("near32", N.PHS_NEAR32)):
        info = None

        def step():
            pl = N.Plan(xy, 2, 1, precision=prec)
            pl.precond_build(m=30, nu=1.0, seed=0)
            w, beta, inf = pl.solve(f, rtol=1e-8)
            pl.eval(w, beta, tg)
            torch.cuda.synchronize()
            pl.close()
            return inf, w, beta

        step()
        t0 = time.perf_counter()
        for _ in range(steps):
            info, w, beta = step()
        ms = (time.perf_counter() - t0) / steps * 1e3
        out[name] = {"ms_per_step": round(ms, 3), **_info_fields(info)}
        sols[name] = (w.cpu().numpy(), beta.cpu().numpy())
    return out, sols


def batch_leg(N, W, torch, n_prob: int, maxit: int = 300, retune: bool = False):
    """Many problems (n log-uniform in [1e3, 2e5], uniform or clustered, k in
    {1..4}, minimal block, 4 right-hand sides each): one batch in mixed
    precision (FP32 FMM, FP64 Krylov with FP64 residual refinement) and the
    same batch in FP64, against the plain FP64 path solving each problem
    alone; all to 1e-8 within maxit, plans and preconditioners included.
    Problems that do not reach 1e-8 (order 4 with ~1e5 nodes or more, whose
    saddle systems are too ill-conditioned for an FP64 operator) are counted
    and listed, not fatal; with `retune` their preconditioner is retuned on
    their own data and the solve repeated."""
    probs = W.batched(n_problems=n_prob)
    dev = torch.device("cuda")
    data = [(torch.as_tensor(p.xy, device=dev), torch.as_tensor(p.f, device=dev), p.k,
             p.precond["m"]) for p in probs]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plans = []
    for xy, f, k, m in data:
        pl = N.Plan(xy, k, -1)
        pl.precond_build(m=m, nu=k / 2.0, seed=0)
        plans.append(pl)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    progress(f"batched: {n_prob} plans and factors in {t_setup:.2f} s")
    batch = N.Batch(plans, [4] * len(plans))
    t1 = time.perf_counter()
    _, infos = batch.solve([f for _, f, _, _ in data], rtol=1e-8, maxit=maxit,
                           precision=N.PHS_MIXED, raise_on_error=False)
    torch.cuda.synchronize()
    t_solve = time.perf_counter() - t1
    res_b = [i.rel_residual for i in infos]
    progress(f"batched: mixed solve {t_solve:.2f} s")
    it32 = sum(i.iters_fp32 for i in infos)
    it64 = sum(i.iters_fp64 for i in infos)
    falls = sum(i.fp64_fallback for i in infos)
    # the same batch in FP64: batching without the precision change
    t1 = time.perf_counter()
    _, infos64 = batch.solve([f for _, f, _, _ in data], rtol=1e-8, maxit=maxit,
                             precision=N.PHS_FP64, raise_on_error=False)
    torch.cuda.synchronize()
    t_solve64 = time.perf_counter() - t1
    res_b64 = [i.rel_residual for i in infos64]
    progress(f"batched: FP64 solve {t_solve64:.2f} s")
    batch.close()
    for pl in plans:
        pl.close()
    t2 = time.perf_counter()
    res_a = []
    for i, (xy, f, k, m) in enumerate(data):
        pl = N.Plan(xy, k, -1)
        pl.precond_build(m=m, nu=k / 2.0, seed=0)
        _, _, info = pl.solve(f, rtol=1e-8, maxit=maxit, raise_on_error=False)
        res_a.append(info.rel_residual)
        pl.close()
        if (i + 1) % 32 == 0:
            progress(f"batched: {i + 1} problems solved alone")
    torch.cuda.synchronize()
    t_alone = time.perf_counter() - t2
    # problems the default preconditioner leaves above 1e-8: retune their
    # preconditioner on their own data (phs_tune_precond) and solve again
    retuned = []
    t3 = time.perf_counter()
    for i, (xy, f, k, m) in enumerate(data):
        if res_b64[i] <= 1e-8 or not retune:
            continue
        pl = N.Plan(xy, k, -1)
        r = pl.tune_precond(f[:, 0].contiguous(), rtol=1e-8, max_evals=6, maxit=400)
        _, _, info = pl.solve(f, rtol=1e-8, maxit=maxit, raise_on_error=False)
        progress(f"batched: problem {i} retuned")
        retuned.append({"problem": i, "n": int(xy.shape[0]), "k": k,
                        "default_rel_residual": res_b64[i], "m": r["m"], "nu": r["nu"],
                        "alpha": round(r["alpha"], 4), "rel_residual": info.rel_residual,
                        "iters": info.iters})
        pl.close()
    torch.cuda.synchronize()
    t_retune = time.perf_counter() - t3
    fixed = sum(1 for r in retuned if r["rel_residual"] <= 1e-8)
    npts = sum(p.n for p in probs)
    ok = lambda r: sum(1 for v in r if v <= 1e-8)
    return {"problems": n_prob, "rhs_per_problem": 4, "points": npts, "maxit": maxit,
            "batched_mixed_s": round(t_setup + t_solve, 4), "batched_setup_s": round(t_setup, 4),
            "batched_solve_s": round(t_solve, 4), "alone_fp64_s": round(t_alone, 4),
            "batched_fp64_s": round(t_setup + t_solve64, 4),
            "batched_fp64_solve_s": round(t_solve64, 4),
            "speedup": round(t_alone / (t_setup + t_solve), 3),
            "speedup_batching_fp64": round(t_alone / (t_setup + t_solve64), 3),
            "speedup_mixed_over_batched_fp64": round(t_solve64 / t_solve, 3),
            "iters_fp32": it32, "iters_fp64": it64, "fp64_fallbacks": falls,
            "at_1e-8_batched": ok(res_b), "at_1e-8_batched_fp64": ok(res_b64),
            "at_1e-8_alone": ok(res_a),
            "at_1e-8_after_retune": (ok(res_b64) + fixed) if retune else None,
            "retune_s": round(t_retune, 3) if retune else None, "retuned": retuned,
            "missed_1e-8": [{"problem": i, "n": probs[i].n, "k": probs[i].k,
                             "rel_residual_batched_fp64": res_b64[i]}
                            for i in range(n_prob) if res_b64[i] > 1e-8],
            "median_rel_residual_batched": float(np.median(res_b)),
            "worst_rel_residual_batched": max(res_b), "worst_rel_residual_alone": max(res_a)}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "bench.py measures one GPU only: the solver runs on a "
                          "single MI355X and has no multi-GPU path",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch
    from paper_2608_11462_amd import native as N
    from paper_2608_11462_amd import workloads as W

    prec = {"fp64": N.PHS_FP64, "mixed": N.PHS_MIXED, "near32": N.PHS_NEAR32}[args.precision]
    pr = W.large_tps(n=args.n)
    dev = torch.device("cuda")
    xy = torch.as_tensor(pr.xy, device=dev)
    f = torch.as_tensor(pr.f, device=dev)
    tg = torch.as_tensor(pr.targets, device=dev)
    torch.cuda.synchronize()

    if args.copy_calibration:
        src = torch.ones(1 << 27, dtype=torch.float64, device=dev)
        dst = torch.mul(src, 2.0)
        torch.cuda.synchronize()
        del src, dst

    phases = {"plan": 0.0, "precond": 0.0, "solve": 0.0, "eval": 0.0}
    last = {}

    def step(record: bool):
        t0 = time.perf_counter()
        pl = N.Plan(xy, 2, 1, precision=prec)
        t1 = time.perf_counter()
        pl.precond_build(m=30, nu=1.0, seed=0)
        t2 = time.perf_counter()
        w, beta, info = pl.solve(f, rtol=1e-8)
        t3 = time.perf_counter()
        s = pl.eval(w, beta, tg)
        torch.cuda.synchronize()
        t4 = time.perf_counter()
        if record:
            phases["plan"] += t1 - t0
            phases["precond"] += t2 - t1
            phases["solve"] += t3 - t2
            phases["eval"] += t4 - t3
            last.update(iters=info.iters, outer=info.outer_refinements,
                        resid=info.rel_residual, L=pl.leaf_level, P=pl.order, R=pl.R,
                        info=info)
            last["leaf"] = pl.tree()[1]
            last["w"], last["beta"] = w, beta
        pl.close()
        return s

    for _ in range(args.warmup):
        step(False)
    progress("warm-up step done")
    torch.cuda.synchronize()
    if not args.no_profile:
        N.profile_enable(2)  # HIP events around the roofline kernels only
        N.profile_read()  # reset
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = {}
    if not args.no_profile:
        prof = N.profile_read()
        N.profile_enable(False)
    ms_per_step = 1e3 * elapsed / args.steps
    n = pr.n

    # matvec throughput on a prebuilt plan (not part of `value`)
    pl = N.Plan(xy, 2, 1)
    v = torch.as_tensor(W.rng_for(17).standard_normal(n), device=dev)
    mv = {}
    for name, p in (("fp64", N.PHS_FP64), ("mixed", N.PHS_MIXED), ("near32", N.PHS_NEAR32)):
        for _ in range(2):
            pl.matvec(v, p)
        torch.cuda.synchronize()
        t = time.perf_counter()
        reps = 10
        for _ in range(reps):
            pl.matvec(v, p)
        torch.cuda.synchronize()
        mv[name] = n / ((time.perf_counter() - t) / reps) / 1e6
    # the FP32 leaf kernel of the mixed matvec, timed with HIP events on its
    # stream (its roofline is reported beside the FP64 step's)
    prof32 = {}
    if not args.no_profile:
        N.profile_enable(2)
        N.profile_read()
        for _ in range(10):
            pl.matvec(v, N.PHS_MIXED)
        torch.cuda.synchronize()
        prof32 = N.profile_read()
        N.profile_enable(False)
    pl.close()
    # the all-pairs P2P kernel of exact-matvec plans (the hybrid solver's
    # operator), FP32 and FP64, on the first N_P2P nodes of the workload:
    # every one of the N_P2P^2 pairs is formed, so the work is known exactly
    if not args.no_profile:
        pd = N.Plan(xy[:N_P2P].contiguous(), 2, 1, matvec=N.PHS_MATVEC_DIRECT)
        vd = v[:N_P2P].contiguous()
        for p in (N.PHS_FP64, N.PHS_MIXED):
            pd.matvec(vd, p)
        torch.cuda.synchronize()
        N.profile_enable(2)
        N.profile_read()
        for _ in range(10):
            for p in (N.PHS_FP64, N.PHS_MIXED):
                pd.matvec(vd, p)
        torch.cuda.synchronize()
        for kname, val in N.profile_read().items():
            if kname in ("direct", "direct_f32"):
                prof32[kname] = val
        N.profile_enable(False)
        pd.close()

    # rooflines from the HIP-event durations of the timed region
    roofs = {}
    # kernel time of the timed steps alone (before the other legs' kernels
    # join the roofline table)
    kernels = {k: {"launches": v[0], "total_ms": round(v[1], 3)}
               for k, v in sorted(prof.items(), key=lambda kv: -kv[1][1])[:12]}
    if prof:
        leaf = last["leaf"].cpu().numpy()
        pairs, m2l_pairs = tree_work(leaf, last["L"], n)
        P, R, m = last["P"], last["R"], 30
        P32 = 15  # FP32 expansion order of the plan
        nnz = n * m - m * (m + 1) // 2
        for kname in ("leaf_eval_f32", "m2l_f32", "direct", "direct_f32"):
            if kname in prof32:
                prof[kname] = prof32[kname]
        models = {
            # kernel: (work per launch, unit, peak, bound)
            "leaf_eval": (pairs * FLOP_PAIR + n * R * 8 * P, "TFLOP/s",
                          FP64_PEAK_TFLOPS, "alu"),
            "leaf_eval_near32": (pairs * FLOP_PAIR + n * R * 8 * P, "TFLOP/s",
                                 FP32_NOPACK_TFLOPS, "alu"),
            # FP32 without packed math: 78.6 TFLOP/s (157.3 with packed FP32)
            "leaf_eval_f32": (pairs * FLOP_PAIR + n * R * 8 * P32, "TFLOP/s",
                              FP32_NOPACK_TFLOPS, "alu"),
            # FP64 M2L runs on the matrix cores (FP64 MFMA peak = vector peak)
            "m2l": (m2l_pairs * R * (4 * (P + 1) ** 2 + 12 * (P + 1)), "TFLOP/s",
                    FP64_PEAK_TFLOPS, "mfma"),
            "m2l_f32": (m2l_pairs * R * (4 * (P32 + 1) ** 2 + 12 * (P32 + 1)), "TFLOP/s",
                        FP32_NOPACK_TFLOPS, "alu"),
            # all-pairs P2P: N_P2P^2 pairs at the near-pair flop count
            "direct": (N_P2P * N_P2P * FLOP_PAIR, "TFLOP/s", FP64_PEAK_TFLOPS, "alu"),
            "direct_f32": (N_P2P * N_P2P * FLOP_PAIR, "TFLOP/s", FP32_NOPACK_TFLOPS, "alu"),
            "vecchia_factor": (n * (2 * (m + 1) ** 3 / 3 + 2 * m * m
                                    + 20 * (m + 1) * (m + 2) / 2), "TFLOP/s",
                               FP64_PEAK_TFLOPS, "alu"),
            # bytes: factor entries (index + value) and three n-vectors
            "precond_u": (nnz * 12 + n * 28, "GB/s", 8000.0, "hbm"),
            "precond_ut": (nnz * 12 + n * 24, "GB/s", 8000.0, "hbm"),
        }
        for kname, (work, unit, peak, bound) in models.items():
            if kname not in prof:
                continue
            launches, total_ms = prof[kname]
            avg_s = total_ms / launches / 1e3
            scale = 1e12 if unit == "TFLOP/s" else 1e9
            ach = work / avg_s / scale
            roofs[kname] = {"kernel": kname, "bound": bound, "achieved": round(ach, 3),
                            "peak": peak, "unit": unit, "frac": round(ach / peak, 4),
                            "traffic": stored_traffic(kname, "large_tps"),
                            "avg_launch_ms": round(avg_s * 1e3, 4), "launches": launches,
                            "work_per_launch": work, "total_ms": round(total_ms, 3)}
    roof = max((r for k, r in roofs.items() if k not in prof32), key=lambda r: r["total_ms"],
               default=None)

    out = {
        "metric": "solve time n=2^20 TPS at 1e-8 rel; FMM matvec Mpts/s; p50/p99 serve latency",
        "value": round(n / (ms_per_step / 1e3) / 1e6, 4),
        "unit": "Mpts/s (nodes solved per second: plan+precond+PCG to 1e-8+beta+10^4-target eval)",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None,
        "dtype": {N.PHS_FP64: "f64", N.PHS_MIXED: "f32 FMM / f64 Krylov",
                  N.PHS_NEAR32: "f64 far field, f32 near field / f64 Krylov"}[prec],
        "data": "synthetic",
        "config": {"workload": "large_tps", "n": n, "k": 2, "poly_degree": 1,
                   "field": "16-mode random Fourier, |kappa|<=8", "targets": int(tg.shape[0]),
                   "precond": "Vecchia/Matern nu=1 alpha=0.35 m=30", "rtol": 1e-8,
                   "precision": args.precision},
        "solve_seconds": round(ms_per_step / 1e3, 4),
        "phase_seconds": {k: round(v / args.steps, 4) for k, v in phases.items()},
        "pcg_iters": last.get("iters"), "outer_refinements": last.get("outer"),
        "rel_residual_fp64": last.get("resid"),
        "plan_seconds_lib": round(last["info"].t_plan, 4) if "info" in last else None,
        "precond_seconds_lib": round(last["info"].t_precond, 4) if "info" in last else None,
        "leaf_level": last.get("L"), "expansion_order": last.get("P"),
        "matvec_mpts_s": {k: round(v, 2) for k, v in mv.items()},
        "serve_p50_ms": None, "serve_p99_ms": None,
        "roofline": roof,
        "rooflines": {k: {kk: v[kk] for kk in ("achieved", "peak", "unit", "frac",
                                               "avg_launch_ms", "work_per_launch")}
                      for k, v in roofs.items()},
        "flop_convention": "near pair 9, L2P 8P per point and density, M2L "
                           "4(P+1)^2 + 12(P+1) per pair and density",
        "kernels": kernels,
    }
    progress(f"{args.steps} timed steps: {ms_per_step:.2f} ms per step")
    checks = None
    if "w" in last and args.n == (1 << 20):
        checks = {"fp64": (last["w"].cpu().numpy(), last["beta"].cpu().numpy())}
    if not args.no_precision_leg:
        pf, sols = precision_leg(N, torch, xy, f, tg)
        out["precision_forms"] = pf
        out["precision_forms"]["fp64"] = {"ms_per_step": round(ms_per_step, 3),
                                          **_info_fields(last["info"])}
        if checks is not None:
            checks.update(sols)
    if not args.no_crossover:
        out["fmm_direct_crossover"] = crossover_leg(N, W, torch)
        progress("crossover leg done")
    if not args.no_tree_leg:
        out["tree_cost"] = tree_leg(N, W, torch)
        progress("tree cost leg done")
    if not args.no_serve and args.serve_requests > 0:
        sv = serve_leg(N, W, torch, args.serve_requests)
        out["serve_p50_ms"], out["serve_p99_ms"] = sv["p50_ms"], sv["p99_ms"]
        out["serving"] = sv
    if args.serve_sweep:
        out["serving_sweep"] = serve_leg(N, W, torch, 512, loads=(0.8, 1.0, 1.2))
    if not args.no_batch and args.batch_problems > 0:
        out["batched"] = batch_leg(N, W, torch, args.batch_problems, retune=args.retune)
    if not args.no_cpu_baseline:
        progress("CPU oracle baseline starts")
        out["cpu_baseline"] = cpu_baseline(checks)
        for name, r in out["cpu_baseline"].get("node_residual_vs_oracle_4096", {}).items():
            if name in out.get("precision_forms", {}):
                out["precision_forms"][name]["node_residual_vs_oracle_4096"] = r
    print(json.dumps(out))


if __name__ == "__main__":
    main()
