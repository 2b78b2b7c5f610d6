"""Thin ctypes binding of libftgcr.so (the C ABI in include/ftgcr.h).

Argument marshalling only: every step of the solve runs in the HIP library.
PyTorch provides device memory (tensors, the workspace) and the stream.  The
library must be built (``python -m paper_2103_07210_amd.build`` or
``__graft_entry__.build()``); there is no fallback path, and loading raises
if it is missing.
"""
from __future__ import annotations

import ctypes
import os
from typing import List, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libftgcr.so")

OK, E_INVALID, E_HIP, E_NOMEM, E_WORKSPACE, E_UNSUPPORTED = 0, -1, -2, -3, -4, -5
FP64, MIXED = 0, 1
PRECOND_NONE, PRECOND_COLUMN = 0, 1
CONVERGED, MAX_STEPS, STAGNATED, BREAKDOWN = 0, 1, 2, 3
METHOD_GCR, METHOD_GMRES = 0, 1
MESH_LATLON, MESH_OCTAHEDRAL = 0, 1
ORDER_AUTO, ORDER_X, ORDER_Z, ORDER_XCD = 0, 1, 2, 3
KMAX = 16
LOG_CAP = 256
NOALLOC_SCRATCH_BYTES = 64 << 20

EXPORTED = ["ftgcr_default_options", "ftgcr_create", "ftgcr_set_options", "ftgcr_get_options",
            "ftgcr_set_stream", "ftgcr_workspace_bytes", "ftgcr_set_workspace", "ftgcr_solve",
            "ftgcr_solve_batch", "ftgcr_destroy", "ftgcr_last_error", "ftgcr_debug_apply_A",
            "ftgcr_debug_apply_Pinv", "ftgcr_kernel_times", "ftgcr_reset_kernel_times", "ftgcr_autotune",
            "ftgcr_autotune_batch", "ftgcr_bw_probe", "ftgcr_solve_noalloc", "ftgcr_get_tiling"]


class FtgcrError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"ftgcr error {code}: {msg}")
        self.code = code


class Grid(ctypes.Structure):
    _fields_ = [("nlon", ctypes.c_int32), ("nlat", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("shell_depth", ctypes.c_double), ("mesh", ctypes.c_int32)]


class Coeffs(ctypes.Structure):
    _fields_ = [("hill_lon", ctypes.c_double), ("hill_lat", ctypes.c_double),
                ("hill_amp", ctypes.c_double), ("hill_width", ctypes.c_double),
                ("decay_z", ctypes.c_double), ("helmholtz", ctypes.c_double)]


class Options(ctypes.Structure):
    _fields_ = [("ft", ctypes.c_int32), ("poll_steps", ctypes.c_int32),
                ("max_steps", ctypes.c_int64), ("inner_tol", ctypes.c_double),
                ("max_refinements", ctypes.c_int32), ("inner_max_steps", ctypes.c_int32),
                ("hist_cap", ctypes.c_int64), ("use_graphs", ctypes.c_int32),
                ("levels_per_block", ctypes.c_int32), ("profile_kernels", ctypes.c_int32),
                ("batch_levels_per_block", ctypes.c_int32), ("method", ctypes.c_int32),
                ("order_stencil", ctypes.c_int32), ("order_dir", ctypes.c_int32)]


class KernelTime(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_int64), ("total_ms", ctypes.c_double)]


class FaultEvent(ctypes.Structure):
    _fields_ = [("step", ctypes.c_int64), ("vec", ctypes.c_int32), ("bit", ctypes.c_int32),
                ("count", ctypes.c_int64), ("start", ctypes.c_int64),
                ("idx", ctypes.c_void_p), ("bits", ctypes.c_void_p)]


class FaultPlan(ctypes.Structure):
    _fields_ = [("n_events", ctypes.c_int32), ("events", ctypes.POINTER(FaultEvent))]


class DetectRec(ctypes.Structure):
    _fields_ = [("step", ctypes.c_int64), ("nu", ctypes.c_int32), ("action", ctypes.c_int32),
                ("rr_old", ctypes.c_double), ("rr_new", ctypes.c_double)]


class Stats(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("detections", ctypes.c_int32),
                ("stagnation_accepts", ctypes.c_int32), ("events_applied", ctypes.c_int32),
                ("steps_executed", ctypes.c_int64), ("steps_accepted", ctypes.c_int64),
                ("steps_wasted", ctypes.c_int64), ("cycles", ctypes.c_int64),
                ("refinements", ctypes.c_int32), ("log_len", ctypes.c_int32),
                ("rhs_norm2", ctypes.c_double), ("rr_final", ctypes.c_double),
                ("rel_res_recursive", ctypes.c_double), ("rel_res_true", ctypes.c_double),
                ("time_ms", ctypes.c_double), ("log_cap", ctypes.c_int32), ("pad_", ctypes.c_int32),
                ("log", ctypes.POINTER(DetectRec)), ("hist_cap", ctypes.c_int64),
                ("hist_len", ctypes.c_int64), ("hist", ctypes.POINTER(ctypes.c_double))]


_lib = None


def load():
    """Load libftgcr.so (after torch, so both use one HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    import torch  # noqa: F401  -- loads the HIP runtime the library binds to
    if not os.path.exists(LIB_PATH):
        raise FtgcrError(E_UNSUPPORTED, f"{LIB_PATH} is not built; run __graft_entry__.build()")
    lib = ctypes.CDLL(LIB_PATH)
    vp, H = ctypes.c_void_p, ctypes.c_void_p
    lib.ftgcr_default_options.argtypes = [ctypes.POINTER(Options)]
    lib.ftgcr_default_options.restype = None
    lib.ftgcr_create.argtypes = [ctypes.POINTER(Grid), ctypes.POINTER(Coeffs), ctypes.c_int, ctypes.c_int,
                                 ctypes.c_int32, vp, ctypes.POINTER(H)]
    lib.ftgcr_create.restype = ctypes.c_int
    lib.ftgcr_set_options.argtypes = [H, ctypes.POINTER(Options)]
    lib.ftgcr_set_options.restype = ctypes.c_int
    lib.ftgcr_get_options.argtypes = [H, ctypes.POINTER(Options)]
    lib.ftgcr_get_options.restype = ctypes.c_int
    lib.ftgcr_set_stream.argtypes = [H, vp]
    lib.ftgcr_set_stream.restype = ctypes.c_int
    lib.ftgcr_workspace_bytes.argtypes = [H]
    lib.ftgcr_workspace_bytes.restype = ctypes.c_size_t
    lib.ftgcr_set_workspace.argtypes = [H, vp, ctypes.c_size_t]
    lib.ftgcr_set_workspace.restype = ctypes.c_int
    lib.ftgcr_solve.argtypes = [H, vp, vp, ctypes.c_double, ctypes.c_int32, ctypes.POINTER(FaultPlan),
                                ctypes.POINTER(Stats)]
    lib.ftgcr_solve.restype = ctypes.c_int
    lib.ftgcr_solve_noalloc.argtypes = lib.ftgcr_solve.argtypes
    lib.ftgcr_solve_noalloc.restype = ctypes.c_int
    lib.ftgcr_solve_batch.argtypes = [ctypes.POINTER(H), ctypes.c_int32, ctypes.POINTER(vp), ctypes.POINTER(vp),
                                      ctypes.POINTER(ctypes.c_double), ctypes.c_int32, ctypes.POINTER(FaultPlan),
                                      ctypes.POINTER(Stats)]
    lib.ftgcr_solve_batch.restype = ctypes.c_int
    lib.ftgcr_destroy.argtypes = [H]
    lib.ftgcr_destroy.restype = None
    lib.ftgcr_last_error.argtypes = [H]
    lib.ftgcr_last_error.restype = ctypes.c_char_p
    lib.ftgcr_debug_apply_A.argtypes = [H, vp, vp]
    lib.ftgcr_debug_apply_A.restype = ctypes.c_int
    lib.ftgcr_debug_apply_Pinv.argtypes = [H, vp, vp]
    lib.ftgcr_debug_apply_Pinv.restype = ctypes.c_int
    lib.ftgcr_kernel_times.argtypes = [H, ctypes.POINTER(KernelTime), ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]
    lib.ftgcr_kernel_times.restype = ctypes.c_int
    lib.ftgcr_reset_kernel_times.argtypes = [H]
    lib.ftgcr_reset_kernel_times.restype = ctypes.c_int
    lib.ftgcr_autotune.argtypes = [H, vp, vp, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]
    lib.ftgcr_autotune.restype = ctypes.c_int
    i32p = ctypes.POINTER(ctypes.c_int32)
    lib.ftgcr_get_tiling.argtypes = [H, i32p, i32p, i32p, i32p]
    lib.ftgcr_get_tiling.restype = ctypes.c_int
    lib.ftgcr_autotune_batch.argtypes = [ctypes.POINTER(H), ctypes.c_int32, ctypes.POINTER(vp), ctypes.POINTER(vp),
                                         ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]
    lib.ftgcr_autotune_batch.restype = ctypes.c_int
    lib.ftgcr_bw_probe.argtypes = [vp, vp, ctypes.c_size_t, ctypes.c_int32, vp, ctypes.POINTER(ctypes.c_double)]
    lib.ftgcr_bw_probe.restype = ctypes.c_int
    _lib = lib
    return lib


def _check(rc: int, handle=None):
    if rc != OK:
        msg = load().ftgcr_last_error(handle)
        raise FtgcrError(rc, msg.decode() if msg else "")


def _grid(pb) -> Grid:
    """Lat-lon problems have nx, ny; octahedral ones N (their O_N)."""
    if hasattr(pb, "N"):
        return Grid(0, pb.N, pb.nz, pb.shell_depth, MESH_OCTAHEDRAL)
    return Grid(pb.nx, pb.ny, pb.nz, pb.shell_depth, MESH_LATLON)


def _coeffs(pb) -> Coeffs:
    return Coeffs(pb.hill_lon, pb.hill_lat, pb.hill_amp, pb.hill_width, pb.decay_z, pb.helmholtz)


class _PlanHolder:
    """ctypes view of a list of events (objects with step, vec, bit, idx,
    start, count, bits attributes); keeps the index arrays alive."""

    def __init__(self, plan):
        plan = list(plan or [])
        self.keep = []
        self.events = (FaultEvent * max(1, len(plan)))()
        for q, ev in enumerate(plan):
            e = self.events[q]
            e.step, e.vec, e.bit = int(ev.step), int(ev.vec), int(ev.bit)
            e.start = int(getattr(ev, "start", 0))
            idx = getattr(ev, "idx", None)
            bits = getattr(ev, "bits", None)
            if idx is not None:
                idx = np.ascontiguousarray(idx, dtype=np.int64)
                self.keep.append(idx)
                e.idx = idx.ctypes.data
                e.count = idx.size
            else:
                e.idx = None
                e.count = int(ev.count)
            if bits is not None:
                bits = np.ascontiguousarray(bits, dtype=np.uint8)
                self.keep.append(bits)
                e.bits = bits.ctypes.data
            else:
                e.bits = None
        self.plan = FaultPlan(len(plan), self.events)


def _stats_out(st: Stats, log, hist) -> dict:
    d = {name: getattr(st, name) for name, _ in Stats._fields_
         if name not in ("pad_", "log", "hist", "log_cap", "hist_cap")}
    d["log"] = [dict(step=log[t].step, nu=log[t].nu, action=log[t].action,
                     rr_old=log[t].rr_old, rr_new=log[t].rr_new) for t in range(st.log_len)]
    d["hist"] = hist[: st.hist_len].copy() if hist is not None else None
    return d


class Solver:
    """One FT-GCR handle on the current device: grid, coefficients,
    precision ('fp64' or 'mixed'), the largest k it will solve with and the
    preconditioner ('column': the vertical tridiagonal part of A; 'none':
    P = I)."""

    def __init__(self, problem, precision: str = "fp64", kmax: int = 4, stream=None, precond: str = "column",
                 **options):
        import torch
        lib = load()
        self.problem = problem
        self.precision = {"fp64": FP64, "mixed": MIXED}[precision]
        self.kmax = kmax
        self.device = torch.device("cuda", torch.cuda.current_device())
        self._stream = stream if stream is not None else torch.cuda.current_stream()
        h = ctypes.c_void_p()
        g, c = _grid(problem), _coeffs(problem)
        self.precond = {"column": PRECOND_COLUMN, "none": PRECOND_NONE}[precond]
        _check(lib.ftgcr_create(ctypes.byref(g), ctypes.byref(c), self.precond, self.precision, kmax,
                                ctypes.c_void_p(self._stream.cuda_stream), ctypes.byref(h)), None)
        self._h = h
        self._ws = None
        if options:
            self.set_options(**options)
        else:
            self._alloc_workspace()

    # -- options / workspace ------------------------------------------------
    def options(self) -> dict:
        o = Options()
        _check(load().ftgcr_get_options(self._h, ctypes.byref(o)), self._h)
        return {name: getattr(o, name) for name, _ in Options._fields_}

    def set_options(self, **kw):
        o = Options()
        _check(load().ftgcr_get_options(self._h, ctypes.byref(o)), self._h)
        for key, val in kw.items():
            if not hasattr(o, key):
                raise KeyError(key)
            setattr(o, key, val)
        _check(load().ftgcr_set_options(self._h, ctypes.byref(o)), self._h)
        self._alloc_workspace()

    def workspace_bytes(self) -> int:
        return int(load().ftgcr_workspace_bytes(self._h))

    def _alloc_workspace(self):
        import torch
        need = self.workspace_bytes()
        if self._ws is None or self._ws.numel() < need:
            self._ws = None
            self._ws = torch.empty(need, dtype=torch.uint8, device=self.device)
        _check(load().ftgcr_set_workspace(self._h, ctypes.c_void_p(self._ws.data_ptr()),
                                          self._ws.numel()), self._h)

    # -- solves -------------------------------------------------------------
    def _dev(self, t):
        import torch
        if not isinstance(t, torch.Tensor):
            t = torch.as_tensor(np.asarray(t, dtype=np.float64))
        t = t.to(device=self.device, dtype=torch.float64).contiguous()
        if t.numel() != self.problem.n:
            raise ValueError(f"expected {self.problem.n} entries, got {t.numel()}")
        return t.view(self.problem.shape)

    def solve(self, rhs, x=None, tol: float = 1e-10, k: int = 3, plan=None,
              log_cap: int = LOG_CAP, hist_cap: int = 0, noalloc: bool = False):
        """Solve A x = rhs; returns (x tensor, stats dict).  x (if given) is
        the initial guess and is overwritten in place when it is already a
        contiguous FP64 device tensor.  noalloc=True calls the
        allocation-free entry point (ftgcr_solve_noalloc: the library's
        device scratch instead of the workspace)."""
        import torch
        lib = load()
        entry = lib.ftgcr_solve_noalloc if noalloc else lib.ftgcr_solve
        rhs_t = self._dev(rhs)
        if x is None:
            x_t = torch.zeros_like(rhs_t)
        else:
            x_t = self._dev(x)
        ph = _PlanHolder(plan)
        log = (DetectRec * max(1, log_cap))()
        hist = np.zeros(max(1, hist_cap))
        st = Stats()
        st.log_cap = log_cap
        st.log = ctypes.cast(log, ctypes.POINTER(DetectRec))
        st.hist_cap = hist_cap
        st.hist = hist.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        lib.ftgcr_set_stream(self._h, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
        _check(entry(self._h, ctypes.c_void_p(rhs_t.data_ptr()), ctypes.c_void_p(x_t.data_ptr()),
                     float(tol), int(k), ctypes.byref(ph.plan) if plan else None, ctypes.byref(st)),
               self._h)
        return x_t, _stats_out(st, log, hist if hist_cap > 0 else None)

    def apply_A(self, x):
        import torch
        x_t = self._dev(x)
        y = torch.empty_like(x_t)
        _check(load().ftgcr_debug_apply_A(self._h, ctypes.c_void_p(x_t.data_ptr()), ctypes.c_void_p(y.data_ptr())),
               self._h)
        return y

    def apply_pinv(self, r):
        import torch
        r_t = self._dev(r)
        e = torch.empty_like(r_t)
        _check(load().ftgcr_debug_apply_Pinv(self._h, ctypes.c_void_p(r_t.data_ptr()),
                                             ctypes.c_void_p(e.data_ptr())), self._h)
        return e

    def autotune(self, rhs, k: int = 3, steps: int = 24) -> int:
        """Time `steps` steps per stencil tiling on this problem and keep the
        fastest (also for later handles of the same grid and precision).
        Returns the chosen levels per block."""
        import torch
        rhs_t = self._dev(rhs)
        scratch = torch.empty_like(rhs_t)
        chosen = ctypes.c_int32()
        _check(load().ftgcr_autotune(self._h, ctypes.c_void_p(rhs_t.data_ptr()),
                                     ctypes.c_void_p(scratch.data_ptr()), int(k), int(steps),
                                     ctypes.byref(chosen)), self._h)
        torch.cuda.synchronize()
        return chosen.value

    def tiling(self) -> dict:
        """The stencil tiling of the next solve: levels per block of the dots
        and direction passes and their block orders (ORDER_X, _Z, _XCD)."""
        v = [ctypes.c_int32() for _ in range(4)]
        _check(load().ftgcr_get_tiling(self._h, *[ctypes.byref(a) for a in v]), self._h)
        return {"levels_per_block": v[0].value, "levels_per_block_dir": v[1].value,
                "order_stencil": v[2].value, "order_dir": v[3].value}

    def kernel_times(self) -> dict:
        """{kernel name: (launches, total ms)} accumulated while profile_kernels is on."""
        buf = (KernelTime * 16)()
        n = ctypes.c_int32()
        _check(load().ftgcr_kernel_times(self._h, buf, 16, ctypes.byref(n)), self._h)
        return {buf[q].name.decode(): (buf[q].launches, buf[q].total_ms) for q in range(min(16, n.value))}

    def reset_kernel_times(self):
        _check(load().ftgcr_reset_kernel_times(self._h), self._h)

    def close(self):
        if getattr(self, "_h", None):
            load().ftgcr_destroy(self._h)
            self._h = None
        self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def solve_batch(solvers: Sequence[Solver], rhs: Sequence, xs: Optional[Sequence] = None,
                tols: Optional[Sequence[float]] = None, k: int = 3, plans: Optional[Sequence] = None,
                log_cap: int = LOG_CAP) -> List:
    """Solve several independent problems with one batched launch sequence.
    Returns (list of x tensors, list of stats dicts)."""
    import torch
    lib = load()
    n = len(solvers)
    rhs_t = [s._dev(r) for s, r in zip(solvers, rhs)]
    xs_t = [torch.zeros_like(r) if xs is None or xs[m] is None else solvers[m]._dev(xs[m])
            for m, r in enumerate(rhs_t)]
    tols = list(tols) if tols is not None else [1e-10] * n
    H = (ctypes.c_void_p * n)(*[s._h for s in solvers])
    R = (ctypes.c_void_p * n)(*[t.data_ptr() for t in rhs_t])
    X = (ctypes.c_void_p * n)(*[t.data_ptr() for t in xs_t])
    T = (ctypes.c_double * n)(*tols)
    holders = [_PlanHolder(p) for p in (plans or [None] * n)]
    P = (FaultPlan * n)(*[hd.plan for hd in holders])
    logs = [(DetectRec * max(1, log_cap))() for _ in range(n)]
    S = (Stats * n)()
    for m in range(n):
        S[m].log_cap = log_cap
        S[m].log = ctypes.cast(logs[m], ctypes.POINTER(DetectRec))
    _check(lib.ftgcr_solve_batch(H, n, R, X, T, int(k), P if plans else None, S), solvers[0]._h)
    return xs_t, [_stats_out(S[m], logs[m], None) for m in range(n)]


def bw_probe(nbytes: int = 1 << 30, reps: int = 5) -> float:
    """HBM copy bandwidth (read + write, GB/s) of the library's streaming
    copy kernel over two fresh device buffers of `nbytes` each."""
    import torch
    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    gbs = ctypes.c_double()
    _check(load().ftgcr_bw_probe(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()),
                                 src.numel() * 8, int(reps),
                                 ctypes.c_void_p(torch.cuda.current_stream().cuda_stream), ctypes.byref(gbs)))
    torch.cuda.synchronize()
    assert torch.equal(src, dst), "bandwidth probe copied wrong data"
    return gbs.value


def autotune_batch(solvers: Sequence[Solver], rhs: Sequence, k: int = 3, steps: int = 24) -> int:
    """Time `steps` batched steps of these members per stencil tiling and
    keep the fastest for later solve_batch calls led by solvers[0].  Returns
    the chosen levels per block."""
    import torch
    lib = load()
    n = len(solvers)
    rhs_t = [s._dev(r) for s, r in zip(solvers, rhs)]
    scratch = [torch.empty_like(r) for r in rhs_t]
    H = (ctypes.c_void_p * n)(*[s._h for s in solvers])
    R = (ctypes.c_void_p * n)(*[t.data_ptr() for t in rhs_t])
    X = (ctypes.c_void_p * n)(*[t.data_ptr() for t in scratch])
    chosen = ctypes.c_int32()
    _check(lib.ftgcr_autotune_batch(H, n, R, X, int(k), int(steps), ctypes.byref(chosen)), solvers[0]._h)
    torch.cuda.synchronize()
    return chosen.value
