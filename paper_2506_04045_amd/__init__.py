"""MI355X (gfx950) solver for similarity-based fuzzy clustering.

Python binding of the C ABI in ``include/fc.h``.  Every function here only
marshals arguments: tensors must already live on the GPU (torch is used for
device memory and streams), and every step of the computation runs in the
HIP kernels of ``libfc.so``.

Problem (P), section 2 of the paper: minimise ||S - U U^T||_F^2 over
row-stochastic U (n x c); the paper's membership matrix is X = U^T.
"""
from __future__ import annotations

import ctypes
import math
from dataclasses import dataclass

import numpy as np
import torch

from . import _native as N

__all__ = ["Solver", "Server", "Info", "objective", "project", "spmm", "gram", "gram_noalloc", "gather_probe", "debug_fail_allocations", "history_records", "spectral_norm",
           "library_path"]

_PREC = {"fp64": N.FC_PREC_FP64, "fp32": N.FC_PREC_FP32, "mixed": N.FC_PREC_MIXED}
_DIAG = {"stored": N.FC_DIAG_STORED, "unit": N.FC_DIAG_UNIT}
_DT = {torch.float64: N.FC_F64, torch.float32: N.FC_F32, torch.float16: N.FC_F16}


def library_path() -> str:
    N.load()
    return N.LIB_PATH


def _stream_ptr(stream) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream)


def _dev(t: torch.Tensor, name: str, dtypes=None) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtypes is not None and t.dtype not in dtypes:
        raise TypeError(f"{name} has dtype {t.dtype}, expected one of {dtypes}")
    return t


class _CsrView:
    """Holds the tensors referenced by an fc_csr so they stay alive."""

    def __init__(self, row_ptr, col_idx, val):
        self.row_ptr = _dev(row_ptr, "row_ptr", (torch.int64,))
        self.col_idx = _dev(col_idx, "col_idx", (torch.int32,))
        self.val = _dev(val, "val", (torch.float64, torch.float32, torch.float16))
        n = self.row_ptr.numel() - 1
        if n < 1:
            raise ValueError("row_ptr must have at least 2 entries")
        if self.col_idx.numel() != self.val.numel():
            raise ValueError("col_idx and val differ in length")
        self.c = N.CSR(n, self.col_idx.numel(), self.row_ptr.data_ptr(),
                       self.col_idx.data_ptr(), self.val.data_ptr(), _DT[self.val.dtype])

    @property
    def n(self) -> int:
        return int(self.c.n)


@dataclass
class Info:
    iter: int
    trials: int
    stop_reason: int
    f: float
    f_prev: float
    L: float
    t: float
    beta: float
    pgrad: float
    pgrad_rel: float

    @staticmethod
    def of(i: N.Info) -> "Info":
        return Info(i.iter, i.trials, i.stop_reason, i.f, i.f_prev, i.L, i.t, i.beta, i.pgrad,
                    i.pgrad_rel)


def _options(c: int, precision: str = "fp32", diag: str = "unit", accelerate: bool = True,
             step: float = 0.0, backtrack: bool = False, L0: float = 0.0, eta: float = 2.0,
             max_iter: int = 100, check_every: int = 16, tol_loss: float = math.nan,
             tol_pgrad: float = 0.0, validate: bool = False,
             norm_estimate: str = "power", reorder="none",
             defer_loss: bool = False, single_pass: bool = False, n=None) -> N.Options:
    opt = N.default_options()
    opt.c = int(c)
    opt.precision = _PREC[precision]
    opt.diag = _DIAG[diag]
    opt.accelerate = int(bool(accelerate))
    opt.step_rule = N.FC_STEP_BACKTRACK if backtrack else N.FC_STEP_FIXED
    opt.step = float(step)
    opt.L0 = float(L0)
    opt.eta = float(eta)
    opt.max_iter = int(max_iter)
    opt.check_every = int(check_every)
    opt.tol_loss = float(tol_loss)
    opt.tol_pgrad = float(tol_pgrad)
    opt.validate = int(bool(validate))
    opt.norm_estimate = {"power": 0, "frobenius": 1}[norm_estimate]
    if isinstance(reorder, str):
        opt.reorder = {"none": 0, "degree": 1}[reorder]
    else:   # a given order: internal row i is the caller's row reorder[i]
        src = reorder.cpu().numpy() if torch.is_tensor(reorder) else reorder
        wide = np.asarray(src, dtype=np.int64)
        if wide.ndim != 1 or (n is not None and wide.shape[0] != n):
            raise ValueError(f"a given order holds the {n} row indices, one each")
        if wide.size and (wide.min() < 0 or wide.max() > np.iinfo(np.int32).max):
            raise ValueError("a given order holds row indices 0..n-1")
        perm = np.ascontiguousarray(wide, dtype=np.int32)
        opt.reorder = N.FC_REORDER_GIVEN
        opt.perm = perm.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        opt._perm_keep = perm   # alive while the options are
    opt.defer_loss = int(bool(defer_loss))
    opt.single_pass = int(bool(single_pass))
    return opt


def history_records(hist: dict, accelerate: bool = True) -> list:
    """Per-iteration records of a solver history (Solver.history): for
    iteration n = 0 (the start) .. K, the loss f(Xbar_n) and its decrease
    f(Xbar_{n-1}) - f(Xbar_n) (None where a loss was not formed: deferred or
    single-pass iterations between read-outs), the accepted step tau_n and
    L_n = 1/tau_n, the trials of the iteration, the gradient-mapping norm
    r_n, and beta_n, the weight that formed the point the iteration stepped
    from: Y_n = Xbar_{n-1} + beta_n (Xbar_{n-1} - Xbar_{n-2}) with t_1 = 1,
    t_{k+1} = (1 + sqrt(1 + 4 t_k^2)) / 2 and beta_n = (t_{n-1} - 1) / t_n
    (Alg. 4; 0 for n <= 2 and for GPA)."""
    def num(x):
        x = float(x)
        return x if math.isfinite(x) else None

    f, tau, trials, r = hist["f"], hist["tau"], hist["trials"], hist["r"]
    out = []
    t_prev, t_cur = 1.0, 1.0   # t_{n-1}, t_n
    for n in range(len(f)):
        rec = {"iter": n, "f": num(f[n])}
        if n == 0:
            out.append(rec)
            continue
        if n >= 2:
            t_prev, t_cur = t_cur, (1.0 + math.sqrt(1.0 + 4.0 * t_cur * t_cur)) / 2.0
        beta = (t_prev - 1.0) / t_cur if (accelerate and n >= 2) else 0.0
        df = (f[n - 1] - f[n]) if (math.isfinite(f[n - 1]) and math.isfinite(f[n])) else math.nan
        rec.update({"df": num(df), "tau": num(tau[n]),
                    "L": num(1.0 / tau[n]) if tau[n] > 0 else None,
                    "beta": beta, "trials": int(trials[n]), "pgrad": num(r[n])})
        out.append(rec)
    return out


class Solver:
    """One solve of problem (P): fc_create / fc_step / fc_solve / fc_get_u.

    reorder: "none" (the caller's numbering), "degree" (the library
    renumbers the articles by descending degree) or an integer array of the
    n row indices (a given order: internal row i is the caller's row
    reorder[i]).  Every form returns iterates in the caller's numbering."""

    def __init__(self, row_ptr, col_idx, val, c: int, U0=None, *, precision: str = "fp32",
                 diag: str = "unit", accelerate: bool = True, step: float = 0.0,
                 backtrack: bool = False, L0: float = 0.0, eta: float = 2.0,
                 max_iter: int = 100, check_every: int = 16, tol_loss: float = math.nan,
                 tol_pgrad: float = 0.0, validate: bool = False, step_schedule=None,
                 norm_estimate: str = "power", reorder="none", defer_loss: bool = False,
                 single_pass: bool = False, stream=None):
        lib = N.load()
        self._csr = _CsrView(row_ptr, col_idx, val)
        self.n, self.c = self._csr.n, int(c)
        self.precision = precision
        self.accelerate = bool(accelerate)
        opt = _options(c, precision, diag, accelerate, step, backtrack, L0, eta, max_iter,
                       check_every, tol_loss, tol_pgrad, validate, norm_estimate, reorder,
                       defer_loss, single_pass, n=self.n)
        self._sched = None
        if step_schedule is not None:
            self._sched = np.ascontiguousarray(step_schedule, dtype=np.float64)
            opt.step_schedule = self._sched.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
            opt.step_schedule_len = int(self._sched.shape[0])
        u0_ptr, u0_dt = None, N.FC_F32
        if U0 is not None:
            U0 = _dev(U0, "U0", (torch.float64, torch.float32))
            if tuple(U0.shape) != (self.n, self.c):
                raise ValueError(f"U0 must be ({self.n}, {self.c})")
            u0_ptr, u0_dt = U0.data_ptr(), _DT[U0.dtype]
        self._stream = stream
        h = ctypes.c_void_p()
        N.check(lib.fc_create(ctypes.byref(self._csr.c), ctypes.byref(opt), u0_ptr, u0_dt,
                              _stream_ptr(stream), ctypes.byref(h)))
        self._h = h

    def _handle(self):
        if self._h is None:
            raise RuntimeError("solver destroyed")
        return self._h

    def step(self, iters: int) -> Info:
        info = N.Info()
        N.check(N.load().fc_step(self._handle(), int(iters), ctypes.byref(info)))
        return Info.of(info)

    def step_profiled(self, iters: int):
        """fc_step_profiled: (Info, per-kernel device milliseconds summed over
        the trials launched)."""
        info = N.Info()
        t = N.KernelTimes()
        N.check(N.load().fc_step_profiled(self._handle(), int(iters), ctypes.byref(info),
                                          ctypes.byref(t)))
        return Info.of(info), dict(fused_ms=t.fused_ms, spmm_ms=t.spmm_ms,
                                   reduce_ms=t.reduce_ms, control_ms=t.control_ms,
                                   launches=t.launches)

    def solve(self) -> Info:
        info = N.Info()
        N.check(N.load().fc_solve(self._handle(), ctypes.byref(info)))
        return Info.of(info)

    def info(self) -> Info:
        return self.step(0)

    def get_u(self, dtype=torch.float32) -> torch.Tensor:
        out = torch.empty(self.n, self.c, dtype=dtype, device="cuda")
        N.check(N.load().fc_get_u(self._handle(), out.data_ptr(), _DT[dtype]))
        return out

    def history(self, cap: int | None = None) -> dict:
        cap = cap or 65536
        f = np.zeros(cap)
        tau = np.zeros(cap)
        trials = np.zeros(cap, dtype=np.int32)
        r = np.zeros(cap)
        cnt = ctypes.c_int32(0)
        N.check(N.load().fc_get_history(self._handle(), cap, f.ctypes.data, tau.ctypes.data,
                                        trials.ctypes.data, r.ctypes.data, ctypes.byref(cnt)))
        k = cnt.value
        return dict(f=f[:k].copy(), tau=tau[:k].copy(), trials=trials[:k].copy(), r=r[:k].copy())

    def write_history_jsonl(self, path: str, cap: int | None = None) -> int:
        """One JSON record per iteration (history_records) written to `path`;
        returns the number of records."""
        import json
        recs = history_records(self.history(cap), self.accelerate)
        with open(path, "w") as fh:
            for r in recs:
                fh.write(json.dumps(r) + "\n")
        return len(recs)

    def get_state(self) -> bytes:
        """Checkpoint (fc_get_state) as a bytes object."""
        size = ctypes.c_size_t(0)
        N.check(N.load().fc_get_state(self._handle(), None, ctypes.byref(size)))
        buf = ctypes.create_string_buffer(size.value)
        N.check(N.load().fc_get_state(self._handle(), buf, ctypes.byref(size)))
        return buf.raw[: size.value]

    def set_state(self, state: bytes) -> None:
        """Restore a checkpoint (fc_set_state)."""
        buf = ctypes.create_string_buffer(state, len(state))
        N.check(N.load().fc_set_state(self._handle(), buf, len(state)))

    def close(self) -> None:
        if self._h is not None:
            N.load().fc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


@dataclass
class Result:
    req_id: int
    status: int
    iter: int
    trials: int
    stop_reason: int
    f: float
    t_submit: float
    t_admit: float
    t_finish: float
    t_setup: float
    t_start: float


def _server_options(max_active, hbm_budget, ticks_per_poll, use_graph, grid_fused=None,
                    grid_spmm=None, solo_max=None, spmm_depth=None) -> N.ServerOpts:
    o = N.default_server_options()
    if solo_max is not None:
        o.solo_max = int(solo_max)
    o.max_active = int(max_active)
    o.hbm_budget = float(hbm_budget)
    o.ticks_per_poll = int(ticks_per_poll)
    o.use_graph = int(bool(use_graph))
    for name, vals in (("grid_fused", grid_fused), ("grid_spmm", grid_spmm),
                       ("spmm_depth", spmm_depth)):
        if vals is not None:
            vals = [int(v) for v in vals]
            if len(vals) != 5:
                raise ValueError(f"{name} needs 5 entries (padded widths 4, 8, 16, 32, 64)")
            getattr(o, name)[:] = vals
    return o


def tune_server(requests, max_active: int = 64, hbm_budget: float = 32.0 * 2**30,
                ticks_per_poll: int = 16, use_graph: bool = False, stream=None,
                solo_max: int | None = None) -> dict:
    """fc_server_tune on sample requests, each a dict with row_ptr, col_idx,
    val, c, U0 (or None) and solver options as Solver takes them.  Returns
    the chosen schedule (ticks_per_poll, use_graph, grid_fused, grid_spmm, spmm_depth:
    keyword arguments of Server), the rate of the final run and the number
    of server runs."""
    lib = N.load()
    base = _server_options(max_active, hbm_budget, ticks_per_poll, use_graph,
                           solo_max=solo_max)
    k = len(requests)
    if k < 1:
        raise ValueError("tune_server needs at least one request")
    views, keep = [], []
    csrs = (N.CSR * k)()
    opts = (N.Options * k)()
    u0s = (ctypes.c_void_p * k)()
    u0_dt = None
    for i, r in enumerate(requests):
        v = _CsrView(r["row_ptr"], r["col_idx"], r["val"])
        views.append(v)
        csrs[i] = v.c
        extra = {key: val for key, val in r.items()
                 if key not in ("row_ptr", "col_idx", "val", "c", "U0")}
        opts[i] = _options(int(r["c"]), **extra)
        U0 = r.get("U0")
        if U0 is not None:
            U0 = _dev(U0, "U0", (torch.float64, torch.float32))
            keep.append(U0)
            if u0_dt is not None and _DT[U0.dtype] != u0_dt:
                raise ValueError("all sample starts must have one dtype")
            u0_dt = _DT[U0.dtype]
            u0s[i] = U0.data_ptr()
    best = N.ServerOpts()
    rate = ctypes.c_double(0.0)
    runs = ctypes.c_int32(0)
    N.check(lib.fc_server_tune(ctypes.byref(base), k, csrs, opts, u0s,
                               N.FC_F32 if u0_dt is None else u0_dt,
                               None if stream is None else int(stream.cuda_stream),
                               ctypes.byref(best), ctypes.byref(rate), ctypes.byref(runs)))
    return dict(ticks_per_poll=int(best.ticks_per_poll), use_graph=bool(best.use_graph),
                grid_fused=list(best.grid_fused), grid_spmm=list(best.grid_spmm),
                spmm_depth=list(best.spmm_depth),
                solves_per_s=float(rate.value), runs=int(runs.value))


class Server:
    """Continuous-batching server (fc_server_*).  Submitted tensors are
    borrowed until the request is released."""

    def __init__(self, max_active: int = 64, hbm_budget: float = 32.0 * 2**30,
                 ticks_per_poll: int = 16, use_graph: bool = False, grid_fused=None,
                 grid_spmm=None, stream=None, solo_max: int | None = None, spmm_depth=None):
        """grid_fused / grid_spmm: the launch table, five workgroups-per-CU
        entries for padded widths 4, 8, 16, 32, 64 (0 = built-in), as
        tune_server returns it.  solo_max: active requests up to which a new
        request runs unbatched on a stream of its own (None = the library's
        default, 4; 0 batches every request).  spmm_depth: the batched sparse
        product's gathers in flight per slot for each padded width (2, 4 or
        8; 0 = built-in 4), a tile shape that changes no result."""
        lib = N.load()
        o = _server_options(max_active, hbm_budget, ticks_per_poll, use_graph, grid_fused,
                            grid_spmm, solo_max, spmm_depth)
        h = ctypes.c_void_p()
        N.check(lib.fc_server_create(ctypes.byref(o), None if stream is None
                                     else int(stream.cuda_stream), ctypes.byref(h)))
        self._h = h
        self._keep = {}

    @staticmethod
    def clock() -> float:
        return float(N.load().fc_server_clock())

    def submit(self, req_id: int, row_ptr, col_idx, val, c: int, U0=None, **options) -> None:
        csr = _CsrView(row_ptr, col_idx, val)
        opt = _options(c, n=csr.n, **options)
        u0_ptr, u0_dt = None, N.FC_F32
        if U0 is not None:
            U0 = _dev(U0, "U0", (torch.float64, torch.float32))
            u0_ptr, u0_dt = U0.data_ptr(), _DT[U0.dtype]
        N.check(N.load().fc_server_submit(self._h, ctypes.byref(csr.c), ctypes.byref(opt),
                                          u0_ptr, u0_dt, int(req_id)))
        self._keep[int(req_id)] = (csr, U0, csr.n, int(c))

    def poll(self, max_results: int = 256, timeout_us: int = 0) -> list:
        buf = (N.Result * max_results)()
        cnt = ctypes.c_int32(0)
        N.check(N.load().fc_server_poll(self._h, buf, max_results, int(timeout_us),
                                        ctypes.byref(cnt)))
        return [Result(r.req_id, r.status, r.iter, r.trials, r.stop_reason, r.f, r.t_submit,
                       r.t_admit, r.t_finish, r.t_setup, r.t_start) for r in buf[: cnt.value]]

    def cancel(self, req_id: int) -> None:
        """Stop a queued or running request (fc_server_cancel); it is reported
        by poll with status FC_ERR_CANCELLED."""
        N.check(N.load().fc_server_cancel(self._h, int(req_id)))

    def get_u(self, req_id: int, dtype=torch.float32) -> torch.Tensor:
        _, _, n, c = self._keep[int(req_id)]
        out = torch.empty(n, c, dtype=dtype, device="cuda")
        N.check(N.load().fc_server_get_u(self._h, int(req_id), out.data_ptr(), _DT[dtype]))
        return out

    def release(self, req_id: int) -> None:
        N.check(N.load().fc_server_release(self._h, int(req_id)))
        self._keep.pop(int(req_id), None)

    def stats(self) -> dict:
        p, a = ctypes.c_int32(), ctypes.c_int32()
        d, b = ctypes.c_int64(), ctypes.c_double()
        N.check(N.load().fc_server_stats(self._h, ctypes.byref(p), ctypes.byref(a),
                                         ctypes.byref(d), ctypes.byref(b)))
        return dict(pending=p.value, active=a.value, done=d.value, bytes_in_use=b.value)

    def close(self) -> None:
        if self._h is not None:
            N.load().fc_server_destroy(self._h)
            self._h = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def objective(row_ptr, col_idx, val, U: torch.Tensor, diag: str = "unit", stream=None) -> float:
    """Structured objective of Alg. 3 (fc_objective)."""
    csr = _CsrView(row_ptr, col_idx, val)
    U = _dev(U, "U", (torch.float64, torch.float32))
    out = ctypes.c_double(0.0)
    N.check(N.load().fc_objective(ctypes.byref(csr.c), _DIAG[diag], U.data_ptr(), _DT[U.dtype],
                                  U.shape[1], _stream_ptr(stream), ctypes.byref(out)))
    return float(out.value)


def project(V: torch.Tensor, out: torch.Tensor | None = None, c: int | None = None,
            stream=None) -> torch.Tensor:
    """Row-wise projection onto the unit simplex (fc_project).  V is (rows, ld)
    and the first c columns of each row are projected."""
    V = _dev(V, "V", (torch.float64, torch.float32))
    if V.dim() != 2:
        raise ValueError("V must be 2-D")
    if out is None:
        out = torch.empty_like(V)
    out = _dev(out, "out", (V.dtype,))
    rows, ld = V.shape
    c = ld if c is None else int(c)
    N.check(N.load().fc_project(V.data_ptr(), out.data_ptr(), _DT[V.dtype], rows, c, ld,
                                _stream_ptr(stream)))
    return out


def spmm(row_ptr, col_idx, val, U: torch.Tensor, diag: str = "unit", stream=None) -> torch.Tensor:
    """Z = S_eff U (fc_spmm)."""
    csr = _CsrView(row_ptr, col_idx, val)
    U = _dev(U, "U", (torch.float64, torch.float32))
    Z = torch.empty_like(U)
    N.check(N.load().fc_spmm(ctypes.byref(csr.c), _DIAG[diag], U.data_ptr(), Z.data_ptr(),
                             _DT[U.dtype], U.shape[1], _stream_ptr(stream)))
    return Z


def gram(U: torch.Tensor, stream=None) -> np.ndarray:
    """G = U^T U in double (fc_gram), returned as a host array."""
    U = _dev(U, "U", (torch.float64, torch.float32))
    n, c = U.shape
    G = np.zeros((c, c))
    N.check(N.load().fc_gram(U.data_ptr(), _DT[U.dtype], n, c, _stream_ptr(stream),
                             G.ctypes.data))
    return G


def gram_noalloc(U: torch.Tensor, G_out: torch.Tensor, stream=None) -> torch.Tensor:
    """G_out = U^T U (fc_gram_noalloc): U (n x c, any row stride) read in
    place, G_out a caller-owned c x c float64 device tensor; asynchronous,
    allocates nothing."""
    if not isinstance(U, torch.Tensor) or not U.is_cuda:
        raise TypeError("U must be a CUDA (HIP) tensor")
    if U.dtype not in (torch.float64, torch.float32):
        raise TypeError(f"U has dtype {U.dtype}, expected float64 or float32")
    if U.dim() != 2 or U.stride(1) != 1 or U.stride(0) < U.shape[1]:
        raise ValueError("U must be 2-D with unit column stride and row stride >= c")
    n, c = U.shape
    if (G_out.device.type != "cuda" or G_out.dtype != torch.float64
            or tuple(G_out.shape) != (c, c) or not G_out.is_contiguous()):
        raise ValueError("G_out must be a contiguous c x c float64 CUDA tensor")
    N.check(N.load().fc_gram_noalloc(U.data_ptr(), _DT[U.dtype], n, c, U.stride(0),
                                     _stream_ptr(stream), G_out.data_ptr()))
    return G_out


def gather_probe(col_idx: torch.Tensor, U: torch.Tensor, wg_per_cu: int = 16, reps: int = 5,
                 stream=None) -> float:
    """Mean device milliseconds of one flat pass that gathers row col_idx[e]
    of U for every e (fc_gather_probe; a memory-system measurement)."""
    col_idx = _dev(col_idx, "col_idx", (torch.int32,))
    U = _dev(U, "U")
    row_bytes = U.shape[1] * U.element_size()
    if U.dim() != 2 or row_bytes not in (32, 64, 128, 256):
        raise ValueError("U must be 2-D with rows of 32, 64, 128 or 256 bytes")
    ms = ctypes.c_double(0.0)
    N.check(N.load().fc_gather_probe(col_idx.data_ptr(), col_idx.numel(), U.data_ptr(),
                                     U.shape[0], row_bytes, wg_per_cu, reps,
                                     _stream_ptr(stream), ctypes.byref(ms)))
    return float(ms.value)


def debug_fail_allocations(after: int) -> None:
    """Test hook (fc_debug_fail_allocations): after `after` more successful
    library allocations every later one fails as out of memory; a negative
    value turns the injection off."""
    N.load().fc_debug_fail_allocations(int(after))


def spectral_norm(row_ptr, col_idx, val, diag: str = "unit", max_iter: int = 1000,
                  rtol: float = 1e-12, stream=None):
    """(||S_eff||_2, power iterations) (fc_spectral_norm)."""
    csr = _CsrView(row_ptr, col_idx, val)
    out = ctypes.c_double(0.0)
    it = ctypes.c_int32(0)
    N.check(N.load().fc_spectral_norm(ctypes.byref(csr.c), _DIAG[diag], int(max_iter),
                                      float(rtol), _stream_ptr(stream), ctypes.byref(out),
                                      ctypes.byref(it)))
    return float(out.value), int(it.value)


def hessian_vector(row_ptr, col_idx, val, U: torch.Tensor, V: torch.Tensor, diag: str = "unit",
                   stream=None) -> torch.Tensor:
    """Hess f(U) V, Theorem 4.1 eq. (hessian) (fc_hessian_vector)."""
    csr = _CsrView(row_ptr, col_idx, val)
    U = _dev(U, "U", (torch.float64, torch.float32))
    V = _dev(V, "V", (U.dtype,))
    if V.shape != U.shape:
        raise ValueError("V must have the shape of U")
    HV = torch.empty_like(U)
    N.check(N.load().fc_hessian_vector(ctypes.byref(csr.c), _DIAG[diag], U.data_ptr(), V.data_ptr(),
                                       HV.data_ptr(), _DT[U.dtype], U.shape[1], _stream_ptr(stream)))
    return HV


def curvature(row_ptr, col_idx, val, U: torch.Tensor, V0: torch.Tensor, krylov: int = 40,
              diag: str = "unit", zero_tol: float = 0.0, stream=None):
    """(lambda_min, V, steps): smallest curvature of f at U over the face
    directions and its Ritz direction (fc_curvature)."""
    csr = _CsrView(row_ptr, col_idx, val)
    U = _dev(U, "U", (torch.float64, torch.float32))
    V0 = _dev(V0, "V0", (U.dtype,))
    if V0.shape != U.shape:
        raise ValueError("V0 must have the shape of U")
    V = torch.empty_like(U)
    lam = ctypes.c_double(0.0)
    steps = ctypes.c_int32(0)
    N.check(N.load().fc_curvature(ctypes.byref(csr.c), _DIAG[diag], U.data_ptr(), V0.data_ptr(),
                                  _DT[U.dtype], U.shape[1], int(krylov), float(zero_tol),
                                  ctypes.byref(lam), V.data_ptr(), ctypes.byref(steps),
                                  _stream_ptr(stream)))
    return float(lam.value), V, int(steps.value)

