"""ctypes wrapper of the FT-GCR CPU oracle -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the CPU-baseline leg of the benchmark
may use this module.  It does not import the GPU package; problems and fault
plans are taken by duck typing (any object with the Problem / FaultEvent
attribute names).

Functions and what pins them (tests/test_oracle_*.py):
  face_weights / apply_A -- closed-form manufactured solutions (second-order
      consistency of the flux form, Eq. (1) operator), symmetry, constant
      null space of the unshifted operator, SPD spectrum on tiny grids;
  hill -- independent chord-length great-circle formula;
  apply_pinv -- dense solves of the vertical tridiagonal blocks extracted
      from the assembled operator;
  solve (Algorithm 1) -- dense LU solutions, right-preconditioned GMRES
      residual norms for a single long cycle, GCR orthogonality invariants,
      and predicted fault outcomes (detected transient fault reproduces the
      fault-free solution bit for bit; x and p faults never reach r);
  solve(method='gmres') (FT-GMRES(k), the same fault layer on restarted
      GMRES) -- per-step residual norms of an independent dense restarted
      GMRES (QR of the power Krylov basis, least squares) over several
      cycles, GCR(k) on one long cycle, dense LU solutions, and predicted
      fault outcomes (x flips caught at the cycle end, overflowing v or
      A z flips at their step, both recovered bit for bit; flips of z are
      consistent with A z and never detected);
  OctOracle (the octahedral reduced Gaussian grid O_N of Section 3) --
      the point counts and equatorial spacings of Table 1, Gauss-Legendre
      nodes and weights against numpy, Euler's formula for the triangulation
      and control areas against the area of the sphere, symmetry, zero row
      sums and SPD spectra of the operator, convergence of the finite-volume
      Laplacian to the spherical-harmonic eigenvalues, the preconditioner
      against dense column solves, and the solvers against dense LU.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libftgcr_oracle.so")

CONVERGED, MAX_STEPS, STAGNATED, BREAKDOWN = 0, 1, 2, 3


class _Problem(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("shell_depth", ctypes.c_double), ("hill_lon", ctypes.c_double),
                ("hill_lat", ctypes.c_double), ("hill_amp", ctypes.c_double),
                ("hill_width", ctypes.c_double), ("decay_z", ctypes.c_double),
                ("helmholtz", ctypes.c_double)]


class _Event(ctypes.Structure):
    _fields_ = [("step", ctypes.c_int64), ("vec", ctypes.c_int32), ("bit", ctypes.c_int32),
                ("count", ctypes.c_int64), ("start", ctypes.c_int64),
                ("idx", ctypes.c_void_p), ("bits", ctypes.c_void_p)]


class _Detect(ctypes.Structure):
    _fields_ = [("step", ctypes.c_int64), ("nu", ctypes.c_int32), ("action", ctypes.c_int32),
                ("rr_old", ctypes.c_double), ("rr_new", ctypes.c_double)]


class _Stats(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("detections", ctypes.c_int32),
                ("stagnation_accepts", ctypes.c_int32), ("events_applied", ctypes.c_int32),
                ("steps_executed", ctypes.c_int64), ("steps_accepted", ctypes.c_int64),
                ("steps_wasted", ctypes.c_int64), ("cycles", ctypes.c_int64),
                ("rhs_norm2", ctypes.c_double), ("rr_final", ctypes.c_double),
                ("rel_res_recursive", ctypes.c_double), ("log_len", ctypes.c_int32),
                ("pad_", ctypes.c_int32), ("hist_len", ctypes.c_int64)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from oracle import build as _build
            _build.build()
        lib = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER(_Problem)
        dp = ctypes.c_void_p
        lib.orc_face_weights.argtypes = [P, dp, dp, dp]
        lib.orc_face_weights.restype = None
        lib.orc_hill.argtypes = [P, ctypes.c_double, ctypes.c_double]
        lib.orc_hill.restype = ctypes.c_double
        lib.orc_apply_A.argtypes = [P, dp, dp, dp, dp, dp]
        lib.orc_apply_A.restype = None
        lib.orc_apply_pinv.argtypes = [P, dp, dp, dp, dp, dp]
        lib.orc_apply_pinv.restype = None
        lib.orc_dot.argtypes = [ctypes.c_int64, dp, dp]
        lib.orc_dot.restype = ctypes.c_double
        lib.orc_solve.argtypes = [P, dp, dp, ctypes.c_double, ctypes.c_int32, ctypes.c_int64,
                                  ctypes.c_int32, ctypes.POINTER(_Event), ctypes.c_int32,
                                  ctypes.POINTER(_Stats), ctypes.POINTER(_Detect), ctypes.c_int32,
                                  dp, ctypes.c_int64]
        lib.orc_solve.restype = ctypes.c_int
        lib.orc_solve_traced.argtypes = lib.orc_solve.argtypes + [dp, dp, ctypes.c_int64]
        lib.orc_solve_traced.restype = ctypes.c_int
        lib.orc_gmres_solve.argtypes = lib.orc_solve.argtypes
        lib.orc_gmres_solve.restype = ctypes.c_int
        lib.orc_solve_pc.argtypes = [P, ctypes.c_int32, ctypes.c_int32] + lib.orc_solve.argtypes[1:]
        lib.orc_solve_pc.restype = ctypes.c_int
        OP = ctypes.POINTER(_OctProblem)
        lib.orc_oct_cells.argtypes = [ctypes.c_int32]
        lib.orc_oct_cells.restype = ctypes.c_int64
        lib.orc_oct_ring_points.argtypes = [ctypes.c_int32, ctypes.c_int32]
        lib.orc_oct_ring_points.restype = ctypes.c_int32
        lib.orc_oct_gauss.argtypes = [ctypes.c_int32, dp, dp]
        lib.orc_oct_gauss.restype = None
        lib.orc_oct_mesh.argtypes = [OP, dp, dp, dp, ctypes.POINTER(ctypes.c_int64)]
        lib.orc_oct_mesh.restype = ctypes.c_int
        lib.orc_oct_apply_A.argtypes = [OP, dp, dp]
        lib.orc_oct_apply_A.restype = ctypes.c_int
        lib.orc_oct_apply_pinv.argtypes = [OP, dp, dp]
        lib.orc_oct_apply_pinv.restype = ctypes.c_int
        lib.orc_oct_solve.argtypes = [OP, dp, dp, ctypes.c_double, ctypes.c_int32, ctypes.c_int64, ctypes.c_int32,
                                      ctypes.c_int32, ctypes.POINTER(_Event), ctypes.c_int32, ctypes.POINTER(_Stats),
                                      ctypes.POINTER(_Detect), ctypes.c_int32, dp, ctypes.c_int64]
        lib.orc_oct_solve.restype = ctypes.c_int
        lib.orc_oct_solve_pc.argtypes = [OP, ctypes.c_int32, ctypes.c_int32, dp, dp, ctypes.c_double, ctypes.c_int32,
                                         ctypes.c_int64, ctypes.c_int32, ctypes.POINTER(_Event), ctypes.c_int32,
                                         ctypes.POINTER(_Stats), ctypes.POINTER(_Detect), ctypes.c_int32, dp,
                                         ctypes.c_int64]
        lib.orc_oct_solve_pc.restype = ctypes.c_int
        lib.orc_set_threads.argtypes = [ctypes.c_int32]
        lib.orc_set_threads.restype = ctypes.c_int
        lib.orc_threads.argtypes = []
        lib.orc_threads.restype = ctypes.c_int32
        _lib = lib
    return _lib


def set_threads(n: int) -> None:
    """Threads for the operator and preconditioner applications; every
    result is bitwise independent of the count."""
    if _load().orc_set_threads(int(n)) != 0:
        raise ValueError("thread count must be >= 1")


def threads() -> int:
    return int(_load().orc_threads())


def _problem(pb) -> _Problem:
    return _Problem(pb.nx, pb.ny, pb.nz, pb.shell_depth, pb.hill_lon, pb.hill_lat,
                    pb.hill_amp, pb.hill_width, pb.decay_z, pb.helmholtz)


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def _vec(a, n) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.float64).reshape(-1)
    if a.size != n:
        raise ValueError(f"expected {n} entries, got {a.size}")
    return a


class _OctProblem(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int32), ("nz", ctypes.c_int32), ("shell_depth", ctypes.c_double),
                ("hill_lon", ctypes.c_double), ("hill_lat", ctypes.c_double), ("hill_amp", ctypes.c_double),
                ("hill_width", ctypes.c_double), ("decay_z", ctypes.c_double), ("helmholtz", ctypes.c_double)]


def _events(plan, keep):
    plan = list(plan or [])
    events = (_Event * max(1, len(plan)))()
    for q, ev in enumerate(plan):
        idx = getattr(ev, "idx", None)
        bits = getattr(ev, "bits", None)
        e = events[q]
        e.step, e.vec, e.bit = int(ev.step), int(ev.vec), int(ev.bit)
        e.start = int(getattr(ev, "start", 0))
        if idx is not None:
            idx = np.ascontiguousarray(idx, dtype=np.int64)
            keep.append(idx)
            e.idx = idx.ctypes.data
            e.count = idx.size
        else:
            e.idx = None
            e.count = int(ev.count)
        if bits is not None:
            bits = np.ascontiguousarray(bits, dtype=np.uint8)
            keep.append(bits)
            e.bits = bits.ctypes.data
        else:
            e.bits = None
    return events, len(plan)


class OctOracle:
    """FP64 reference of the octahedral O_N operator, its column
    preconditioner and FT-GCR(k) / FT-GMRES(k) on it.  `problem` has N, nz
    and the coefficient fields of the lat-lon problems (shell_depth,
    hill_lon, hill_lat, hill_amp, hill_width, decay_z, helmholtz)."""

    def __init__(self, problem):
        self.problem = problem
        pb = problem
        self._c = _OctProblem(pb.N, pb.nz, pb.shell_depth, pb.hill_lon, pb.hill_lat, pb.hill_amp,
                              pb.hill_width, pb.decay_z, pb.helmholtz)
        lib = _load()
        self.cells = int(lib.orc_oct_cells(pb.N))

    @property
    def n(self) -> int:
        return self.cells * self.problem.nz

    def ring_points(self):
        return np.array([_load().orc_oct_ring_points(self.problem.N, j) for j in range(2 * self.problem.N)])

    def gauss(self):
        m = 2 * self.problem.N
        mu, w = np.empty(m), np.empty(m)
        _load().orc_oct_gauss(self.problem.N, _ptr(mu), _ptr(w))
        return mu, w

    def mesh(self):
        """Longitude, latitude and control area of every point, and the
        number of edges of the triangulation."""
        m = self.cells
        lon, lat, area = np.empty(m), np.empty(m), np.empty(m)
        ne = ctypes.c_int64()
        if _load().orc_oct_mesh(ctypes.byref(self._c), _ptr(lon), _ptr(lat), _ptr(area), ctypes.byref(ne)) != 0:
            raise ValueError("bad O_N problem")
        return lon, lat, area, int(ne.value)

    def apply_A(self, x) -> np.ndarray:
        x = _vec(x, self.n)
        y = np.empty(self.n)
        if _load().orc_oct_apply_A(ctypes.byref(self._c), _ptr(x), _ptr(y)) != 0:
            raise ValueError("bad O_N problem")
        return y

    def apply_pinv(self, r) -> np.ndarray:
        r = _vec(r, self.n)
        e = np.empty(self.n)
        if _load().orc_oct_apply_pinv(ctypes.byref(self._c), _ptr(r), _ptr(e)) != 0:
            raise ValueError("bad O_N problem")
        return e

    def dense_matrix(self) -> np.ndarray:
        n = self.n
        if n > 4096:
            raise ValueError("dense assembly is for tiny grids")
        m = np.empty((n, n))
        unit = np.zeros(n)
        for c in range(n):
            unit[c] = 1.0
            m[:, c] = self.apply_A(unit)
            unit[c] = 0.0
        return m

    def dot(self, a, b) -> float:
        return _load().orc_dot(self.n, _ptr(_vec(a, self.n)), _ptr(_vec(b, self.n)))

    def solve(self, rhs, x0=None, tol: float = 1e-10, k: int = 3, max_steps: int = 100000, ft: bool = True,
              plan=None, log_cap: int = 4096, hist_cap: Optional[int] = None, method: str = "gcr",
              precond: str = "column"):
        """FT-GCR(k) or FT-GMRES(k) on the O_N problem, with the column
        preconditioner or none (precond 'none': P = I); returns (x, stats,
        detection log, residual history) as Oracle.solve."""
        if method not in ("gcr", "gmres") or precond not in ("column", "none"):
            raise ValueError("method is 'gcr' or 'gmres', precond 'column' or 'none'")
        rhs = _vec(rhs, self.n)
        x = np.zeros(self.n) if x0 is None else _vec(x0, self.n).copy()
        keep = []
        events, nev = _events(plan, keep)
        if hist_cap is None:
            hist_cap = min(max_steps, 1 << 20)
        hist = np.zeros(max(1, hist_cap))
        log = (_Detect * max(1, log_cap))()
        st = _Stats()
        rc = _load().orc_oct_solve_pc(ctypes.byref(self._c), 1 if precond == "column" else 0,
                                      {"gcr": 0, "gmres": 1}[method], _ptr(rhs), _ptr(x), float(tol), int(k),
                                      int(max_steps), 1 if ft else 0, events, nev, ctypes.byref(st),
                                      log, int(log_cap), _ptr(hist), int(hist_cap))
        if rc != 0:
            raise ValueError("oracle rejected the arguments")
        stats = {name: getattr(st, name) for name, _ in _Stats._fields_ if name != "pad_"}
        dlog = [dict(step=log[t].step, nu=log[t].nu, action=log[t].action,
                     rr_old=log[t].rr_old, rr_new=log[t].rr_new) for t in range(st.log_len)]
        return x, stats, dlog, hist[: st.hist_len].copy()

    def true_residual(self, x, rhs) -> float:
        r = self.apply_A(x) - _vec(rhs, self.n)
        return float(np.sqrt(self.dot(r, r) / self.dot(rhs, rhs)))


class Oracle:
    """FP64 reference implementation of the operator, preconditioner and
    FT-GCR(k) on one problem."""

    def __init__(self, problem):
        self.problem = problem
        self._c = _problem(problem)
        self._w = None

    @property
    def n(self) -> int:
        return self.problem.nx * self.problem.ny * self.problem.nz

    @property
    def shape(self):
        return (self.problem.nz, self.problem.ny, self.problem.nx)

    def face_weights(self):
        if self._w is None:
            pb = self.problem
            wx = np.empty((pb.nz, pb.ny, pb.nx))
            wy = np.empty((pb.nz, pb.ny + 1, pb.nx))
            wz = np.empty((pb.nz + 1, pb.ny, pb.nx))
            _load().orc_face_weights(ctypes.byref(self._c), _ptr(wx), _ptr(wy), _ptr(wz))
            self._w = (wx, wy, wz)
        return self._w

    def hill(self, lon: float, lat: float) -> float:
        return _load().orc_hill(ctypes.byref(self._c), lon, lat)

    def apply_A(self, x) -> np.ndarray:
        wx, wy, wz = self.face_weights()
        x = _vec(x, self.n)
        y = np.empty(self.n)
        _load().orc_apply_A(ctypes.byref(self._c), _ptr(wx), _ptr(wy), _ptr(wz), _ptr(x), _ptr(y))
        return y.reshape(self.shape)

    def apply_pinv(self, r) -> np.ndarray:
        wx, wy, wz = self.face_weights()
        r = _vec(r, self.n)
        e = np.empty(self.n)
        _load().orc_apply_pinv(ctypes.byref(self._c), _ptr(wx), _ptr(wy), _ptr(wz), _ptr(r), _ptr(e))
        return e.reshape(self.shape)

    def dot(self, a, b) -> float:
        a = _vec(a, self.n)
        b = _vec(b, self.n)
        return _load().orc_dot(self.n, _ptr(a), _ptr(b))

    def dense_matrix(self) -> np.ndarray:
        """A assembled column by column from apply_A (tiny grids only)."""
        n = self.n
        if n > 4096:
            raise ValueError("dense assembly is for tiny grids")
        m = np.empty((n, n))
        unit = np.zeros(n)
        for c in range(n):
            unit[c] = 1.0
            m[:, c] = self.apply_A(unit).reshape(-1)
            unit[c] = 0.0
        return m

    def solve(self, rhs, x0=None, tol: float = 1e-10, k: int = 3, max_steps: int = 100000,
              ft: bool = True, plan: Optional[Sequence] = None, log_cap: int = 4096,
              hist_cap: Optional[int] = None, trace: bool = False, method: str = "gcr",
              precond: str = "column"):
        """Run FT-GCR(k) (method 'gcr') or FT-GMRES(k) ('gmres') with the
        column preconditioner or none (precond 'none': P = I).  Returns
        (x, stats dict, detection log, rr history).  With trace=True (GCR,
        column preconditioner) the stats also hold the per-step
        orthogonality diagnostics 'cos_r_ap' and 'cos_ap' (see
        orc_solve_traced)."""
        if method not in ("gcr", "gmres") or precond not in ("column", "none") or \
                (trace and (method != "gcr" or precond != "column")):
            raise ValueError("method is 'gcr' or 'gmres', precond 'column' or 'none'; trace is for GCR")
        rhs = _vec(rhs, self.n)
        x = np.zeros(self.n) if x0 is None else _vec(x0, self.n).copy()
        plan = list(plan or [])
        keep = []
        events = (_Event * max(1, len(plan)))()
        for q, ev in enumerate(plan):
            idx = getattr(ev, "idx", None)
            bits = getattr(ev, "bits", None)
            e = events[q]
            e.step, e.vec, e.bit = int(ev.step), int(ev.vec), int(ev.bit)
            e.start = int(getattr(ev, "start", 0))
            if idx is not None:
                idx = np.ascontiguousarray(idx, dtype=np.int64)
                keep.append(idx)
                e.idx = idx.ctypes.data
                e.count = idx.size
            else:
                e.idx = None
                e.count = int(ev.count)
            if bits is not None:
                bits = np.ascontiguousarray(bits, dtype=np.uint8)
                keep.append(bits)
                e.bits = bits.ctypes.data
            else:
                e.bits = None
        if hist_cap is None:
            hist_cap = min(max_steps, 1 << 20)
        hist = np.zeros(max(1, hist_cap))
        log = (_Detect * max(1, log_cap))()
        st = _Stats()
        cos_r_ap = np.zeros(max(1, hist_cap)) if trace else None
        cos_ap = np.zeros(max(1, hist_cap)) if trace else None
        if precond == "none":
            rc = _load().orc_solve_pc(
                ctypes.byref(self._c), 0, 1 if method == "gmres" else 0, _ptr(rhs), _ptr(x), float(tol), int(k),
                int(max_steps), 1 if ft else 0, events, len(plan), ctypes.byref(st), log, int(log_cap),
                _ptr(hist), int(hist_cap))
        elif method == "gmres":
            rc = _load().orc_gmres_solve(
                ctypes.byref(self._c), _ptr(rhs), _ptr(x), float(tol), int(k), int(max_steps),
                1 if ft else 0, events, len(plan), ctypes.byref(st), log, int(log_cap),
                _ptr(hist), int(hist_cap))
        else:
            rc = _load().orc_solve_traced(
                ctypes.byref(self._c), _ptr(rhs), _ptr(x), float(tol), int(k), int(max_steps),
                1 if ft else 0, events, len(plan), ctypes.byref(st), log, int(log_cap),
                _ptr(hist), int(hist_cap), _ptr(cos_r_ap) if trace else None,
                _ptr(cos_ap) if trace else None, int(hist_cap) if trace else 0)
        if rc != 0:
            raise ValueError("oracle rejected the arguments")
        stats = {name: getattr(st, name) for name, _ in _Stats._fields_ if name != "pad_"}
        if trace:
            stats["cos_r_ap"] = cos_r_ap[: st.hist_len].copy()
            stats["cos_ap"] = cos_ap[: st.hist_len].copy()
        dlog = [dict(step=log[t].step, nu=log[t].nu, action=log[t].action,
                     rr_old=log[t].rr_old, rr_new=log[t].rr_new) for t in range(st.log_len)]
        return x.reshape(self.shape), stats, dlog, hist[: st.hist_len].copy()

    def true_residual(self, x, rhs) -> float:
        """||A x - R|| / ||R||."""
        r = self.apply_A(x).reshape(-1) - _vec(rhs, self.n)
        return float(np.sqrt(self.dot(r, r) / self.dot(rhs, rhs)))
