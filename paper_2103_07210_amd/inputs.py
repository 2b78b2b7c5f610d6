"""Seeded synthetic inputs for FT-GCR runs: problems, right-hand sides and
bit-flip fault plans.

This module holds data generation only -- no arithmetic of the method.  Both
the GPU path and the CPU oracle consume what it produces, so it is the one
piece of Python the two sides share.  Random numbers come from NumPy's PCG64
(``numpy.random.default_rng``) with the seeds listed per configuration.

The paper's own test problem (potential flow over a hill on octahedral
meshes, Section 3, Eq. (3)) needs a terrain-following operator and meshes the
paper does not give; the synthetic hill-on-sphere operator below stands in for
it.  The paper injects faults into e = P^{-1}(r) right after preconditioning
(Section 3); the plans here target x, r, the current direction p or its image
A p at a given executed step, as the campaign configurations ask.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

VEC_X, VEC_R, VEC_P, VEC_AP, VEC_E = 0, 1, 2, 3, 4
VEC_NAMES = {"x": VEC_X, "r": VEC_R, "p": VEC_P, "ap": VEC_AP, "e": VEC_E}


@dataclasses.dataclass(frozen=True)
class Problem:
    """Grid and coefficient parameters of the synthetic hill-on-sphere operator.

    c(lon, lat, zeta) = 1 + hill_amp * h(lon, lat) * exp(-zeta / decay_z),
    h = exp(-(gc / hill_width)^2), gc = great-circle distance to the hill
    centre; A = A0 + helmholtz * diag(A0).
    """
    nx: int
    ny: int
    nz: int
    shell_depth: float = 1.0
    hill_lon: float = math.pi / 2
    hill_lat: float = math.pi / 6
    hill_amp: float = 0.5
    hill_width: float = 0.35
    decay_z: float = 0.3
    helmholtz: float = 1e-3

    @property
    def n(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)


@dataclasses.dataclass(frozen=True)
class OctProblem:
    """The octahedral reduced Gaussian grid O_N of the paper's experiments
    (Section 3, Table 1) with nz levels: 4N(N+9) points per level, fields
    [nz][points]; coefficients as for Problem."""
    N: int
    nz: int
    shell_depth: float = 1.0
    hill_lon: float = math.pi / 2
    hill_lat: float = math.pi / 6
    hill_amp: float = 0.5
    hill_width: float = 0.35
    decay_z: float = 0.3
    helmholtz: float = 1e-3

    @property
    def points(self) -> int:
        return 4 * self.N * (self.N + 9)

    @property
    def n(self) -> int:
        return self.points * self.nz

    @property
    def shape(self):
        return (self.nz, self.points)


@dataclasses.dataclass
class FaultEvent:
    """XOR `bit` (or per-entry `bits`) into entries of one working vector
    during executed step `step` (1-based): x, r, p^nu, L(p^nu) at the start
    of the step; e = P^-1(r) right after the step's preconditioner (only if
    the step passes its tests).  `idx` lists flat canonical indices; if it
    is None the entries are the range [start, start+count)."""
    step: int
    vec: int
    bit: int = 62
    idx: Optional[np.ndarray] = None
    start: int = 0
    count: int = 1
    bits: Optional[np.ndarray] = None

    def __post_init__(self):
        if isinstance(self.vec, str):
            self.vec = VEC_NAMES[self.vec]
        if self.idx is not None:
            self.idx = np.ascontiguousarray(self.idx, dtype=np.int64)
            self.count = int(self.idx.size)
        if self.bits is not None:
            self.bits = np.ascontiguousarray(self.bits, dtype=np.uint8)

    def indices(self) -> np.ndarray:
        if self.idx is not None:
            return self.idx
        return np.arange(self.start, self.start + self.count, dtype=np.int64)


Plan = List[FaultEvent]

# --- the five workload configurations ---------------------------------------

# the paper's O160 with its 51 levels (Table 1) and a small octahedral case
O160 = OctProblem(160, 51)
O40 = OctProblem(40, 51)

C1 = Problem(64, 32, 8)
C2 = Problem(256, 128, 32)
C3 = Problem(512, 256, 64)
C5 = Problem(1024, 512, 96)
C4_SIZES = ((64, 32, 8), (128, 64, 16), (192, 96, 24), (256, 128, 32))

SEEDS = {"c1_rhs": 1, "c1_plan": 101, "c2_rhs": 2, "c2_plan0": 1000,
         "c3_rhs": 3, "c4_table": 4, "c4_rhs0": 4000, "c4_plan0": 4100,
         "c5_rhs": 5, "c5_plan": 501, "paper_plan0": 6000}


def rhs(problem: Problem, seed: int) -> np.ndarray:
    """R ~ U[-1, 1] in canonical [nz][ny][nx] order (FP64)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-1.0, 1.0, problem.n).reshape(problem.shape)


def single_flip_plan(problem: Problem, seed: int, step: int = 5, vec: str = "r",
                     bit: int = 62) -> Plan:
    """One event: flip `bit` of one uniformly drawn entry of `vec` at `step`."""
    rng = np.random.default_rng(seed)
    at = int(rng.integers(0, problem.n))
    return [FaultEvent(step=step, vec=vec, bit=bit, idx=np.array([at]))]


def campaign_plans(problem: Problem, count: int = 200, seed0: int = 1000,
                   max_step: int = 20, bit_max: int = 63) -> List[Plan]:
    """Fault campaign, one event per solve: step U{1..max_step}, vector
    U{x, r, p, Ap}, size U{one entry; 1% of entries drawn without replacement;
    a contiguous block of 10% of entries}, one bit U{0..bit_max} applied to
    every corrupted entry."""
    plans = []
    n = problem.n
    for m in range(count):
        rng = np.random.default_rng(seed0 + m)
        step = int(rng.integers(1, max_step + 1))
        vec = int(rng.integers(0, 4))
        size_kind = int(rng.integers(0, 3))
        bit = int(rng.integers(0, bit_max + 1))
        if size_kind == 0:
            ev = FaultEvent(step, vec, bit, idx=np.array([int(rng.integers(0, n))]))
        elif size_kind == 1:
            cnt = int(math.ceil(0.01 * n))
            ev = FaultEvent(step, vec, bit, idx=np.sort(rng.choice(n, cnt, replace=False)))
        else:
            cnt = int(math.ceil(0.1 * n))
            ev = FaultEvent(step, vec, bit, start=int(rng.integers(0, n - cnt + 1)), count=cnt)
        plans.append([ev])
    return plans


def block_plan(problem: Problem, step: int = 10, vec: str = "r", fraction: float = 0.1,
               bit: int = 62, seed: int = 501) -> Plan:
    """One contiguous-block event covering `fraction` of the entries."""
    rng = np.random.default_rng(seed)
    cnt = int(math.ceil(fraction * problem.n))
    return [FaultEvent(step=step, vec=vec, bit=bit,
                       start=int(rng.integers(0, problem.n - cnt + 1)), count=cnt)]


def process_entries(problem: Problem, procs: int, rank: int) -> np.ndarray:
    """Canonical indices of the entries one of `procs` processes would own
    under a horizontal decomposition into bands of whole columns (column
    index j * nx + i, or the O_N point index, split into `procs` contiguous
    ranges, all levels)."""
    ncols = problem.points if isinstance(problem, OctProblem) else problem.nx * problem.ny
    lo = (ncols * rank) // procs
    hi = (ncols * (rank + 1)) // procs
    cols = np.arange(lo, hi, dtype=np.int64)
    return (cols[None, :] + ncols * np.arange(problem.nz, dtype=np.int64)[:, None]).ravel()


# The two readings of which bit a flip hits (the paper does not say):
# "uniform" draws it from all 64 bits of the binary64 pattern; "finite"
# leaves out bit 62, the top exponent bit, whose flip takes a value in
# [1, 2) to Inf or NaN and a value below 1 in magnitude to one above 2^1023
# (whose square overflows), so that the corrupted entries stay finite and
# their squares mostly so.
BIT_READINGS = {"uniform": tuple(range(64)), "finite": tuple(range(62)) + (63,)}


def paper_plans(problem: Problem, count: int, prob: float = 0.02, data_loss: float = 0.01,
                procs: int = 36, max_events: int = 10, horizon: int = 1000, seed0: int = SEEDS["paper_plan0"],
                bit_max: int = 63, bits: str = "") -> List[Plan]:
    """The paper's fault model (Section 3), one plan per run: after the
    preconditioner of every executed step a fault event happens with
    probability `prob`, at most `max_events` per run; an event hits one
    process drawn at random (one of `procs` bands of whole columns) and
    flips one random bit in each of ceil(data_loss * N) distinct entries of
    that process' share of e = P^-1(r) (all of its entries when the share is
    smaller): U{0..bit_max}, or uniform over BIT_READINGS[bits] when `bits`
    names a reading (the same random draws, mapped onto that set).  Steps
    are drawn up to `horizon`; events past the end of a run are not
    applied."""
    choices = np.array(BIT_READINGS[bits] if bits else range(bit_max + 1), dtype=np.uint8)
    plans = []
    n = problem.n
    cnt = max(1, int(math.ceil(data_loss * n)))
    for m in range(count):
        rng = np.random.default_rng(seed0 + m)
        hits = np.nonzero(rng.random(horizon) < prob)[0][:max_events] + 1
        plan: Plan = []
        for step in hits.tolist():
            own = process_entries(problem, procs, int(rng.integers(0, procs)))
            idx = own if cnt >= own.size else np.sort(rng.choice(own, cnt, replace=False))
            flip = choices[rng.integers(0, choices.size, idx.size)]
            plan.append(FaultEvent(step=int(step), vec=VEC_E, bit=0, idx=idx.astype(np.int64), bits=flip))
        plans.append(plan)
    return plans


@dataclasses.dataclass
class EnsembleMember:
    problem: Problem
    rhs_seed: int
    plan: Plan


def ensemble(count: int = 64, seed: int = 4, faulty_fraction: float = 0.1,
             sizes: Sequence = C4_SIZES, max_step: int = 20) -> List[EnsembleMember]:
    """Batched ensemble: grid sizes drawn from `sizes`, hill centre uniform on
    the sphere's lon/lat box, amplitude U[0.2, 1.0]; round(faulty_fraction *
    count) members get one single-entry flip of bit 62 in r at U{1..max_step}."""
    rng = np.random.default_rng(seed)
    members = []
    faulty = set(rng.choice(count, int(round(faulty_fraction * count)), replace=False).tolist())
    for m in range(count):
        nx, ny, nz = sizes[int(rng.integers(0, len(sizes)))]
        pb = Problem(nx, ny, nz,
                     hill_lon=float(rng.uniform(0.0, 2 * math.pi)),
                     hill_lat=float(rng.uniform(-math.pi / 2, math.pi / 2)),
                     hill_amp=float(rng.uniform(0.2, 1.0)))
        plan: Plan = []
        if m in faulty:
            prng = np.random.default_rng(SEEDS["c4_plan0"] + m)
            plan = [FaultEvent(step=int(prng.integers(1, max_step + 1)), vec=VEC_R, bit=62,
                               idx=np.array([int(prng.integers(0, pb.n))]))]
        members.append(EnsembleMember(pb, SEEDS["c4_rhs0"] + m, plan))
    return members
