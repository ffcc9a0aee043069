"""Thin ctypes binding of libphs.so (argument marshalling only).

Every step of the computation runs in the HIP library; PyTorch only provides
device memory (tensors whose data pointers are handed to the C ABI) and the
current HIP stream.  Importing this module does not load the library; the
first call does, and raises if the library has not been built.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass
from pathlib import Path

import torch

LIB_PATH = Path(__file__).resolve().parent / "libphs.so"

PHS_FP64, PHS_MIXED, PHS_NEAR32 = 0, 1, 2
PHS_MATVEC_FMM, PHS_MATVEC_DIRECT = 0, 1
PHS_RANGE_NORMALIZED, PHS_RANGE_USER = 0, 1

STATUS = {
    0: "PHS_OK", 1: "PHS_ERR_INVALID_ARGUMENT", 2: "PHS_ERR_DUPLICATE_POINTS",
    3: "PHS_ERR_UNISOLVENT", 4: "PHS_ERR_NOT_CONVERGED", 5: "PHS_ERR_BREAKDOWN",
    6: "PHS_ERR_OUT_OF_MEMORY", 7: "PHS_ERR_DEVICE", 8: "PHS_ERR_NOT_READY",
}

EXPORTS = ("phs_plan", "phs_matvec", "phs_precond_build", "phs_solve", "phs_eval",
           "phs_plan_info", "phs_plan_tree", "phs_precond_export", "phs_precond_apply",
           "phs_plan_destroy", "phs_batch_create", "phs_batch_solve", "phs_batch_destroy",
           "phs_server_create", "phs_server_submit", "phs_server_step", "phs_server_poll",
           "phs_server_memory", "phs_server_destroy",
           "phs_tune_precond", "phs_autotune_plan",
           "phs_direct_sum", "phs_direct_sum_noalloc", "phs_last_error", "phs_memory_stats",
           "phs_profile_enable", "phs_profile_read", "phs_set_graphs")
PHS_REQ_QUEUED, PHS_REQ_ACTIVE, PHS_REQ_DONE, PHS_REQ_FAILED = 0, 1, 2, 3


class PlanOpts(C.Structure):
    _fields_ = [("k", C.c_int32), ("poly_degree", C.c_int32), ("precision", C.c_int32),
                ("fmm_tol", C.c_double), ("leaf_size", C.c_int32),
                ("expansion_order", C.c_int32), ("matvec", C.c_int32)]


class PrecondOpts(C.Structure):
    _fields_ = [("m", C.c_int32), ("nu", C.c_double), ("range", C.c_double),
                ("range_units", C.c_int32), ("seed", C.c_uint64)]


class SolveOpts(C.Structure):
    _fields_ = [("rtol", C.c_double), ("maxit", C.c_int32), ("check_every", C.c_int32),
                ("precision", C.c_int32)]


class ServerOpts(C.Structure):
    _fields_ = [("hbm_budget", C.c_int64), ("max_active", C.c_int32), ("precision", C.c_int32),
                ("rtol", C.c_double), ("maxit", C.c_int32)]


class Request(C.Structure):
    _fields_ = [("xy", C.c_void_p), ("f", C.c_void_p), ("targets", C.c_void_p),
                ("n", C.c_int64), ("m", C.c_int64), ("k", C.c_int32),
                ("poly_degree", C.c_int32), ("precond", PrecondOpts), ("w", C.c_void_p),
                ("beta", C.c_void_p), ("values", C.c_void_p)]


class RequestInfo(C.Structure):
    _fields_ = [("state", C.c_int32), ("status", C.c_int32), ("iters", C.c_int32),
                ("rel_residual", C.c_double), ("t_submit", C.c_double),
                ("t_admit", C.c_double), ("t_done", C.c_double), ("bytes", C.c_int64)]


class SolveInfo(C.Structure):
    _fields_ = [("iters", C.c_int32), ("outer_refinements", C.c_int32),
                ("rel_residual", C.c_double), ("t_solve", C.c_double),
                ("iters_fp32", C.c_int32), ("iters_fp64", C.c_int32),
                ("fp64_fallback", C.c_int32), ("reserved", C.c_int32),
                ("t_plan", C.c_double), ("t_precond", C.c_double)]


class TuneOpts(C.Structure):
    _fields_ = [("max_evals", C.c_int32), ("maxit", C.c_int32), ("rtol", C.c_double),
                ("m_min", C.c_int32), ("m_max", C.c_int32)]


class TuneResult(C.Structure):
    _fields_ = [("m", C.c_int32), ("nu", C.c_double), ("alpha", C.c_double),
                ("seconds", C.c_double), ("iters", C.c_int32), ("rel_residual", C.c_double),
                ("evals", C.c_int32), ("default_seconds", C.c_double),
                ("default_iters", C.c_int32)]


class AutotuneOpts(C.Structure):
    _fields_ = [("matvec_tol", C.c_double), ("precision", C.c_int32), ("reps", C.c_int32),
                ("seed", C.c_uint64)]


class AutotuneResult(C.Structure):
    _fields_ = [("matvec", C.c_int32), ("leaf_size", C.c_int32),
                ("expansion_order", C.c_int32), ("candidates", C.c_int32),
                ("matvec_seconds", C.c_double), ("rel_error", C.c_double)]


class PHSError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status
        self.name = STATUS.get(status, str(status))


_lib = None


def lib() -> C.CDLL:
    global _lib
    if _lib is None:
        if not LIB_PATH.exists():
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2608_11462_amd.build`")
        L = C.CDLL(str(LIB_PATH))
        vp, i32, i64, dp = C.c_void_p, C.c_int32, C.c_int64, C.c_void_p
        L.phs_plan.argtypes = [dp, i64, C.POINTER(PlanOpts), vp, C.POINTER(vp)]
        L.phs_matvec.argtypes = [vp, dp, dp, i32, i32, vp]
        L.phs_precond_build.argtypes = [vp, C.POINTER(PrecondOpts), vp]
        L.phs_solve.argtypes = [vp, dp, i32, C.POINTER(SolveOpts), dp, dp,
                                C.POINTER(SolveInfo), vp]
        L.phs_eval.argtypes = [vp, dp, dp, i32, dp, i64, dp, vp]
        L.phs_plan_info.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                    C.POINTER(i32), C.POINTER(i32), C.POINTER(i32),
                                    C.POINTER(i32), C.POINTER(C.c_double)]
        L.phs_plan_tree.argtypes = [vp, dp, dp, vp]
        L.phs_precond_export.argtypes = [vp, dp, dp, dp, dp, vp]
        L.phs_precond_apply.argtypes = [vp, dp, dp, vp]
        L.phs_plan_destroy.argtypes = [vp]
        L.phs_plan_destroy.restype = None
        L.phs_batch_create.argtypes = [C.POINTER(vp), i32, C.POINTER(i32), vp, C.POINTER(vp)]
        L.phs_batch_solve.argtypes = [vp, C.POINTER(vp), C.POINTER(vp), C.POINTER(vp),
                                      C.POINTER(SolveOpts), C.POINTER(SolveInfo), vp]
        L.phs_batch_destroy.argtypes = [vp]
        L.phs_batch_destroy.restype = None
        L.phs_server_create.argtypes = [C.POINTER(ServerOpts), vp, C.POINTER(vp)]
        L.phs_server_submit.argtypes = [vp, C.POINTER(Request), C.POINTER(i64)]
        L.phs_server_step.argtypes = [vp, C.POINTER(i32), C.POINTER(i32)]
        L.phs_server_poll.argtypes = [vp, i64, C.POINTER(RequestInfo)]
        L.phs_server_memory.argtypes = [vp, C.POINTER(i64), C.POINTER(i64)]
        L.phs_server_destroy.argtypes = [vp]
        L.phs_server_destroy.restype = None
        L.phs_last_error.restype = C.c_char_p
        L.phs_memory_stats.argtypes = [C.POINTER(i64)] * 4
        L.phs_direct_sum.argtypes = [i32, dp, i64, dp, dp, i64, dp, vp]
        L.phs_tune_precond.argtypes = [vp, dp, C.POINTER(TuneOpts), C.POINTER(TuneResult), vp]
        L.phs_autotune_plan.argtypes = [dp, i64, i32, i32, C.POINTER(AutotuneOpts),
                                        C.POINTER(PlanOpts), C.POINTER(AutotuneResult), vp]
        L.phs_direct_sum_noalloc.argtypes = [i32, dp, i64, dp, dp, i64, dp, vp]
        L.phs_profile_enable.argtypes = [i32]
        L.phs_profile_enable.restype = None
        L.phs_set_graphs.argtypes = [i32]
        L.phs_set_graphs.restype = None
        L.phs_profile_read.argtypes = [vp, C.POINTER(i64), C.POINTER(C.c_double), i32]
        L.phs_profile_read.restype = i32
        for name in ("phs_plan", "phs_matvec", "phs_precond_build", "phs_solve", "phs_eval",
                     "phs_plan_info", "phs_plan_tree", "phs_precond_export",
                     "phs_precond_apply", "phs_batch_create", "phs_batch_solve",
                     "phs_server_create", "phs_server_submit", "phs_server_step",
                     "phs_server_poll", "phs_server_memory", "phs_memory_stats",
                     "phs_direct_sum", "phs_direct_sum_noalloc", "phs_tune_precond",
                     "phs_autotune_plan"):
            getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def _check(status: int, allow=()) -> int:
    if status != 0 and status not in allow:
        raise PHSError(status, lib().phs_last_error().decode())
    return status


def _stream() -> C.c_void_p:
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t: torch.Tensor, name: str) -> C.c_void_p:
    if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous float64 CUDA tensor")
    return C.c_void_p(t.data_ptr())


def _cols(t: torch.Tensor) -> torch.Tensor:
    """n x nrhs tensor -> column-major storage (nrhs, n) contiguous."""
    if t.dim() == 1:
        return t.contiguous()
    return t.t().contiguous()


@dataclass
class Info:
    iters: int
    outer_refinements: int
    rel_residual: float
    t_solve: float
    status: str
    iters_fp32: int = 0
    iters_fp64: int = 0
    fp64_fallback: int = 0
    t_plan: float = 0.0
    t_precond: float = 0.0


def _info(i: SolveInfo, st: int) -> Info:
    return Info(i.iters, i.outer_refinements, i.rel_residual, i.t_solve,
                STATUS.get(st, str(st)), i.iters_fp32, i.iters_fp64, i.fp64_fallback,
                i.t_plan, i.t_precond)


def autotune_plan(xy: torch.Tensor, k: int, degree: int = -1, matvec_tol: float = 1e-12,
                  precision: int = PHS_FP64, reps: int = 0, seed: int = 0):
    """Pick matvec kind, leaf size and expansion order for these nodes (see
    phs_autotune_plan).  Returns (plan keyword arguments, report dict)."""
    xy = xy.contiguous()
    best = PlanOpts()
    r = AutotuneResult()
    o = AutotuneOpts(matvec_tol, precision, reps, seed)
    _check(lib().phs_autotune_plan(_dev(xy, "xy"), xy.shape[0], k, degree, C.byref(o),
                                   C.byref(best), C.byref(r), _stream()))
    kw = {"degree": best.poly_degree, "precision": best.precision, "leaf_size": best.leaf_size,
          "expansion_order": best.expansion_order, "matvec": best.matvec}
    return kw, {k2: getattr(r, k2) for k2, _ in AutotuneResult._fields_}


def direct_sum(k: int, xy: torch.Tensor, q: torch.Tensor, targets: torch.Tensor) -> torch.Tensor:
    """out[t] = sum_j q_j phi(|targets_t - xy_j|) by all-pairs summation (FP64,
    coordinates as given)."""
    xy, q, tg = xy.contiguous(), q.contiguous(), targets.contiguous()
    out = torch.empty(tg.shape[0], dtype=torch.float64, device=q.device)
    _check(lib().phs_direct_sum(k, _dev(xy, "xy"), xy.shape[0], _dev(q, "q"),
                                _dev(tg, "targets"), tg.shape[0], _dev(out, "out"), _stream()))
    return out


def direct_sum_noalloc(k: int, xy: torch.Tensor, q: torch.Tensor, targets: torch.Tensor,
                       out: torch.Tensor) -> torch.Tensor:
    """direct_sum into a caller-provided `out` through the entry point that
    allocates no device memory (its partial sums use the library's static
    device scratch)."""
    xy, q, tg = xy.contiguous(), q.contiguous(), targets.contiguous()
    if out.numel() != tg.shape[0]:
        raise ValueError("out must hold one value per target")
    _check(lib().phs_direct_sum_noalloc(k, _dev(xy, "xy"), xy.shape[0], _dev(q, "q"),
                                        _dev(tg, "targets"), tg.shape[0], _dev(out, "out"),
                                        _stream()))
    return out


def memory_stats():
    """(allocations, device_mallocs, bytes_in_use, bytes_held) of the library's
    device pool."""
    a, m, u, b = C.c_int64(), C.c_int64(), C.c_int64(), C.c_int64()
    _check(lib().phs_memory_stats(C.byref(a), C.byref(m), C.byref(u), C.byref(b)))
    return a.value, m.value, u.value, b.value


class Plan:
    """A PHS interpolation plan over fixed nodes (device-resident)."""

    def __init__(self, xy: torch.Tensor, k: int, degree: int = -1, precision: int = PHS_FP64,
                 fmm_tol: float = 0.0, leaf_size: int = 0, expansion_order: int = 0,
                 matvec: int = PHS_MATVEC_FMM):
        xy = xy.contiguous()
        _dev(xy, "xy")
        if xy.dim() != 2 or xy.shape[1] != 2:
            raise ValueError("xy must be n x 2")
        self.n = xy.shape[0]
        self.k = k
        opts = PlanOpts(k, degree, precision, fmm_tol, leaf_size, expansion_order, matvec)
        h = C.c_void_p()
        _check(lib().phs_plan(C.c_void_p(xy.data_ptr()), self.n, C.byref(opts), _stream(),
                              C.byref(h)))
        self._h = h
        c = (C.c_double * 2)()
        sc = C.c_double()
        S, R, L, P = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
        th = C.c_double()
        _check(lib().phs_plan_info(h, c, C.byref(sc), C.byref(S), C.byref(R), C.byref(L),
                                   C.byref(P), C.byref(th)))
        self.center = (c[0], c[1])
        self.scale = sc.value
        self.tree_half_width = th.value
        self.S, self.R, self.leaf_level, self.order = S.value, R.value, L.value, P.value

    # -- kernel matvec ---------------------------------------------------
    def matvec(self, v: torch.Tensor, precision: int = PHS_FP64) -> torch.Tensor:
        vc = _cols(v)
        nrhs = 1 if v.dim() == 1 else v.shape[1]
        y = torch.empty_like(vc)
        _check(lib().phs_matvec(self._h, _dev(vc, "v"), _dev(y, "y"), nrhs, precision,
                                _stream()))
        return y if v.dim() == 1 else y.t()

    # -- preconditioner --------------------------------------------------
    def precond_build(self, m: int = 0, nu: float = 0.0, range_: float = 0.0,
                      range_units: int = PHS_RANGE_NORMALIZED, seed: int = 0) -> None:
        o = PrecondOpts(m, nu, range_, range_units, seed)
        _check(lib().phs_precond_build(self._h, C.byref(o), _stream()))

    def tune_precond(self, f: torch.Tensor, rtol: float = 1e-8, max_evals: int = 0,
                     maxit: int = 0, m_min: int = 0, m_max: int = 0) -> dict:
        """Search (m, nu, alpha) for this plan and values f (see phs_tune_precond);
        the plan keeps the best preconditioner."""
        o = TuneOpts(max_evals, maxit, rtol, m_min, m_max)
        r = TuneResult()
        _check(lib().phs_tune_precond(self._h, _dev(f.contiguous(), "f"), C.byref(o), C.byref(r),
                                      _stream()))
        return {k: getattr(r, k) for k, _ in TuneResult._fields_}

    def precond_export(self, m: int):
        dev = torch.device("cuda")
        rank = torch.empty(self.n, dtype=torch.int32, device=dev)
        nbr = torch.empty(self.n * m, dtype=torch.int32, device=dev)
        coef = torch.empty(self.n * m, dtype=torch.float64, device=dev)
        diag = torch.empty(self.n, dtype=torch.float64, device=dev)
        _check(lib().phs_precond_export(self._h, C.c_void_p(rank.data_ptr()),
                                        C.c_void_p(nbr.data_ptr()), C.c_void_p(coef.data_ptr()),
                                        C.c_void_p(diag.data_ptr()), _stream()))
        return rank, nbr.view(self.n, m), coef.view(self.n, m), diag

    def precond_apply(self, r: torch.Tensor) -> torch.Tensor:
        r = r.contiguous()
        z = torch.empty_like(r)
        _check(lib().phs_precond_apply(self._h, _dev(r, "r"), _dev(z, "z"), _stream()))
        return z

    # -- solve / evaluate ---------------------------------------------------
    def solve(self, f: torch.Tensor, rtol: float = 1e-8, maxit: int = 0, check_every: int = 0,
              precision: int = -1, raise_on_error: bool = True):
        fc = _cols(f)
        nrhs = 1 if f.dim() == 1 else f.shape[1]
        w = torch.empty_like(fc)
        beta = torch.empty(nrhs * self.S, dtype=torch.float64, device=fc.device)
        o = SolveOpts(rtol, maxit, check_every, precision)
        inf = SolveInfo()
        st = lib().phs_solve(self._h, _dev(fc, "f"), nrhs, C.byref(o), _dev(w, "w"),
                             _dev(beta, "beta"), C.byref(inf), _stream())
        if raise_on_error:
            _check(st)
        info = _info(inf, st)
        if f.dim() == 1:
            return w, beta, info
        return w.view(nrhs, self.n).t(), beta.view(nrhs, self.S).t(), info

    def eval(self, w: torch.Tensor, beta: torch.Tensor, targets: torch.Tensor) -> torch.Tensor:
        wc, bc = _cols(w), _cols(beta)
        nrhs = 1 if w.dim() == 1 else w.shape[1]
        tg = targets.contiguous()
        m = tg.shape[0]
        out = torch.empty(nrhs * m, dtype=torch.float64, device=wc.device)
        _check(lib().phs_eval(self._h, _dev(wc, "w"), _dev(bc, "beta"), nrhs, _dev(tg, "targets"),
                              m, _dev(out, "out"), _stream()))
        return out if w.dim() == 1 else out.view(nrhs, m).t()

    def tree(self):
        dev = torch.device("cuda")
        order = torch.empty(self.n, dtype=torch.int32, device=dev)
        leaf = torch.empty(self.n, dtype=torch.int32, device=dev)
        _check(lib().phs_plan_tree(self._h, C.c_void_p(order.data_ptr()),
                                   C.c_void_p(leaf.data_ptr()), _stream()))
        return order, leaf

    def close(self) -> None:
        if getattr(self, "_h", None):
            lib().phs_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Several plans (and several right-hand sides per plan) solved together:
    every PCG step is one launch over all systems still iterating."""

    def __init__(self, plans: list, nrhs: list | None = None):
        self.plans = list(plans)
        self.nrhs = list(nrhs) if nrhs is not None else [1] * len(self.plans)
        hs = (C.c_void_p * len(self.plans))(*[p._h.value for p in self.plans])
        rs = (C.c_int32 * len(self.plans))(*self.nrhs)
        h = C.c_void_p()
        _check(lib().phs_batch_create(hs, len(self.plans), rs, _stream(), C.byref(h)))
        self._h = h

    def solve(self, fs: list, rtol: float = 1e-8, maxit: int = 0, check_every: int = 0,
              precision: int = -1, raise_on_error: bool = True):
        """fs[i]: n_i (one RHS) or n_i x nrhs_i tensor for plan i.  Returns a
        list of (w, beta) in the same shapes and a list of Info per plan."""
        np_ = len(self.plans)
        fc = [_cols(f) for f in fs]
        ws = [torch.empty_like(f) for f in fc]
        bs = [torch.empty(r * p.S, dtype=torch.float64, device=f.device)
              for f, r, p in zip(fc, self.nrhs, self.plans)]
        for f, p, r in zip(fc, self.plans, self.nrhs):
            _dev(f, "f")
            if f.numel() != p.n * r:
                raise ValueError("right-hand side shape does not match the plan")
        fp = (C.c_void_p * np_)(*[f.data_ptr() for f in fc])
        wp = (C.c_void_p * np_)(*[w.data_ptr() for w in ws])
        bp = (C.c_void_p * np_)(*[b.data_ptr() for b in bs])
        o = SolveOpts(rtol, maxit, check_every, precision)
        infs = (SolveInfo * np_)()
        st = lib().phs_batch_solve(self._h, fp, wp, bp, C.byref(o), infs, _stream())
        if raise_on_error:
            _check(st)
        out = []
        for f, w, b, p, r in zip(fs, ws, bs, self.plans, self.nrhs):
            if f.dim() == 1:
                out.append((w, b))
            else:
                out.append((w.view(r, p.n).t(), b.view(r, p.S).t()))
        infos = [_info(i, st) for i in infs]
        return out, infos

    def close(self) -> None:
        if getattr(self, "_h", None):
            lib().phs_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def n_monomials(k: int, degree: int) -> int:
    d = degree if degree >= 0 else ((k + 1) // 2 - 1 if k % 2 else k // 2)
    return (d + 1) * (d + 2) // 2


class Server:
    """Request loop with continuous batching (see phs_server_* in phs.h).  The
    binding keeps each request's tensors alive until it is done or failed."""

    def __init__(self, hbm_budget: int = 0, max_active: int = 0, precision: int = PHS_FP64,
                 rtol: float = 1e-8, maxit: int = 0):
        o = ServerOpts(hbm_budget, max_active, precision, rtol, maxit)
        h = C.c_void_p()
        _check(lib().phs_server_create(C.byref(o), _stream(), C.byref(h)))
        self._h = h
        self._t = {}

    def submit(self, xy: torch.Tensor, f: torch.Tensor, k: int, degree: int = -1,
               targets: torch.Tensor | None = None, m: int = 0, nu: float = 0.0,
               range_: float = 0.0, range_units: int = PHS_RANGE_NORMALIZED,
               seed: int = 0) -> int:
        xy, f = xy.contiguous(), f.contiguous()
        _dev(xy, "xy")
        _dev(f, "f")
        n = xy.shape[0]
        nt = 0 if targets is None else targets.shape[0]
        tg = targets.contiguous() if nt else None
        w = torch.empty(n, dtype=torch.float64, device=xy.device)
        beta = torch.empty(n_monomials(k, degree), dtype=torch.float64, device=xy.device)
        vals = torch.empty(max(nt, 1), dtype=torch.float64, device=xy.device)
        req = Request(xy.data_ptr(), f.data_ptr(), tg.data_ptr() if nt else None, n, nt, k,
                      degree, PrecondOpts(m, nu, range_, range_units, seed), w.data_ptr(),
                      beta.data_ptr(), vals.data_ptr())
        rid = C.c_int64()
        _check(lib().phs_server_submit(self._h, C.byref(req), C.byref(rid)))
        self._t[rid.value] = (xy, f, tg, w, beta, vals[:nt])
        return rid.value

    def step(self):
        a, q = C.c_int32(), C.c_int32()
        _check(lib().phs_server_step(self._h, C.byref(a), C.byref(q)))
        return a.value, q.value

    def poll(self, rid: int) -> RequestInfo:
        inf = RequestInfo()
        _check(lib().phs_server_poll(self._h, rid, C.byref(inf)))
        return inf

    def result(self, rid: int):
        """(w, beta, values) of a request (valid once it is done)."""
        t = self._t[rid]
        return t[3], t[4], t[5]

    def memory(self):
        u, p = C.c_int64(), C.c_int64()
        _check(lib().phs_server_memory(self._h, C.byref(u), C.byref(p)))
        return u.value, p.value

    def close(self) -> None:
        if getattr(self, "_h", None):
            lib().phs_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def set_graphs(on: bool) -> None:
    """PCG iterations replayed from HIP graphs, or launched directly (the default)."""
    lib().phs_set_graphs(int(bool(on)))


def profile_enable(on=True) -> None:
    """on: False/0 off, True/1 every kernel, 2 only the kernels the roofline
    figures use (leaf, M2L, Vecchia factor and KNN, preconditioner apply)."""
    lib().phs_profile_enable(int(on))


def profile_read(cap: int = 256) -> dict:
    names = (C.c_char * 48 * cap)()
    launches = (C.c_int64 * cap)()
    ms = (C.c_double * cap)()
    k = lib().phs_profile_read(C.cast(names, C.c_void_p), launches, ms, cap)
    out = {}
    for i in range(k):
        out[bytes(names[i]).split(b"\0", 1)[0].decode()] = (launches[i], ms[i])
    return out
