"""Pins of the oracle's octahedral reduced Gaussian grid O_N (the paper's
mesh family, Section 3 and Table 1) and of the node-centred finite-volume
operator on it:

* Table 1: 4N(N+9) points per level times 51 levels reproduces every printed
  point count, and the equatorial ring (4N + 16 points) reproduces every
  printed equatorial resolution on a sphere of radius 6371 km;
* ring latitudes and weights: numpy's Gauss-Legendre rule;
* the triangulation: Euler's formula for a sphere with the two polar caps
  open (V - E + F = 0, F = 2V - 40), and the control areas summing to the
  area of its triangles computed independently here;
* the operator: symmetric, zero row sums of the unshifted part (A 1 =
  sigma/(1+sigma) diag(A)), SPD with the smallest eigenvalue at least
  sigma min(diag A0) (A0 is positive semidefinite), and convergence of A0 / area to the spherical-harmonic
  eigenvalues l(l+1) for zonal and longitude-dependent harmonics;
* the preconditioner: dense solves of the column blocks cut from the
  assembled A; the solvers: dense LU, and a detected transient fault
  reproducing the fault-free run bit for bit (Section 3).
"""
import csv
import math
import os
from types import SimpleNamespace as NS

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_table_1_octahedral.csv")


def _problem(N, nz, amp=0.5, helmholtz=1e-3, lon=math.pi / 2, lat=math.pi / 6):
    return NS(N=N, nz=nz, shell_depth=1.0, hill_lon=lon, hill_lat=lat, hill_amp=amp, hill_width=0.35,
              decay_z=0.3, helmholtz=helmholtz)


def _rows():
    with open(GOLDEN) as f:
        return list(csv.DictReader(l for l in f if not l.startswith("#")))


def test_table_1_point_counts_and_equatorial_spacing(oracle_mod):
    rows = _rows()
    assert len(rows) == 5
    for r in rows:
        N = int(r["N"])
        o = oracle_mod.OctOracle(_problem(N, 1))
        pts = o.ring_points()
        assert o.cells * int(r["levels"]) == int(r["points"]), r
        assert pts.sum() == o.cells
        i = np.concatenate([np.arange(1, N + 1), np.arange(N, 0, -1)])
        assert np.array_equal(pts, 4 * i + 16)
        dx = 2 * math.pi * 6371.0 / pts[N]   # the equatorial ring
        half = 0.05 if "." in r["dx_eq_km"] else 0.5   # printed to 0.1 or to 1 km
        assert abs(dx - float(r["dx_eq_km"])) <= half, (r, dx)


@pytest.mark.parametrize("N", [2, 5, 16, 40])
def test_gauss_legendre_matches_numpy(oracle_mod, N):
    mu, w = oracle_mod.OctOracle(_problem(N, 1)).gauss()
    ref_mu, ref_w = np.polynomial.legendre.leggauss(2 * N)
    np.testing.assert_allclose(mu, ref_mu, rtol=0, atol=1e-14)
    np.testing.assert_allclose(w, ref_w, rtol=1e-11)


def _triangle_area_sum(lon, lat, rings):
    """Area of the open-capped inscribed polyhedron, from its triangles
    (re-derived here: each strip between rings of n and n2 points has n + n2
    triangles whose vertices are found by the same eastward walk)."""
    p = np.stack([np.cos(lat) * np.cos(lon), np.cos(lat) * np.sin(lon), np.sin(lat)], 1)
    first = np.concatenate([[0], np.cumsum(rings)])
    total, count = 0.0, 0
    for j in range(len(rings) - 1):
        n, n2 = rings[j], rings[j + 1]
        a = b = 0
        while a < n or b < n2:
            if a < n and (b >= n2 or (a + 1) * n2 <= (b + 1) * n):
                t = (first[j] + a % n, first[j] + (a + 1) % n, first[j + 1] + b % n2)
                a += 1
            else:
                t = (first[j] + a % n, first[j + 1] + b % n2, first[j + 1] + (b + 1) % n2)
                b += 1
            total += 0.5 * np.linalg.norm(np.cross(p[t[1]] - p[t[0]], p[t[2]] - p[t[0]]))
            count += 1
    return total, count


@pytest.mark.parametrize("N", [3, 8, 20])
def test_triangulation_and_control_areas(oracle_mod, N):
    o = oracle_mod.OctOracle(_problem(N, 1))
    lon, lat, area, nedge = o.mesh()
    rings = o.ring_points()
    tri_area, nface = _triangle_area_sum(lon, lat, rings)
    V = o.cells
    assert nface == 2 * V - rings[0] - rings[-1]
    assert V - nedge + nface == 0   # Euler characteristic of a sphere with two holes
    assert abs(area.sum() - tri_area) <= 1e-12 * tri_area
    assert area.min() > 0
    assert tri_area < 4 * math.pi


@pytest.mark.parametrize("N,nz", [(2, 3), (3, 4)])
def test_operator_symmetric_spd_and_null_space(oracle_mod, N, nz):
    o = oracle_mod.OctOracle(_problem(N, nz, amp=0.8, lat=0.3))
    m = o.dense_matrix()
    scale = np.abs(m).max()
    assert np.abs(m - m.T).max() <= 1e-14 * scale
    sigma = 1e-3
    d = np.diag(m)
    np.testing.assert_allclose(m @ np.ones(o.n), sigma / (1 + sigma) * d, rtol=1e-9, atol=1e-13 * scale)
    ev = np.linalg.eigvalsh(0.5 * (m + m.T))
    # A0 is positive semidefinite (cotangent stiffness plus vertical
    # diffusion; some cotangent weights are negative, so not by Gershgorin),
    # hence A = A0 + sigma D0 >= sigma D0 and lambda_min >= sigma min(D0)
    assert ev.min() >= sigma / (1 + sigma) * d.min() * (1 - 1e-9)


@pytest.mark.parametrize("name,ev", [("Y1", 2.0), ("Y11", 2.0), ("Y22", 6.0), ("Y32", 12.0)])
def test_laplacian_converges_to_spherical_harmonic_eigenvalues(oracle_mod, name, ev):
    """c = 1, no shift, one level: A0 phi / (control area) -> l(l+1) phi on
    |lat| <= 60 degrees, for zonal and longitude-dependent harmonics."""
    f = {"Y1": lambda la, lo: np.sin(la), "Y11": lambda la, lo: np.cos(la) * np.cos(lo),
         "Y22": lambda la, lo: np.cos(la) ** 2 * np.cos(2 * lo),
         "Y32": lambda la, lo: np.cos(la) ** 2 * np.sin(la) * np.sin(2 * lo)}[name]
    errs = []
    for N in (8, 16, 32):
        o = oracle_mod.OctOracle(_problem(N, 1, amp=0.0, helmholtz=1e-300))
        lon, lat, area, _ = o.mesh()
        phi = f(lat, lon)
        y = o.apply_A(phi) / area
        mask = np.abs(lat) <= math.pi / 3
        errs.append(np.max(np.abs(y[mask] - ev * phi[mask])) / np.max(np.abs(ev * phi)))
    assert errs[-1] <= 2e-2, errs
    assert errs[1] < errs[0] / 1.3 and errs[2] < errs[1] / 1.3, errs


def test_vertical_part_matches_closed_form(oracle_mod):
    """A field constant on every level and cos(pi zeta) in height: only the
    vertical faces carry flux, and A0 phi / (area dz) -> (pi / H)^2 phi."""
    errs = []
    for nz in (8, 16, 32):
        o = oracle_mod.OctOracle(_problem(4, nz, amp=0.0, helmholtz=1e-300))
        _, _, area, _ = o.mesh()
        zeta = (np.arange(nz) + 0.5) / nz
        phi = np.repeat(np.cos(math.pi * zeta), o.cells)
        y = o.apply_A(phi) / (np.tile(area, nz) / nz)
        errs.append(np.max(np.abs(y - math.pi ** 2 * phi)) / math.pi ** 2)
    assert errs[2] < errs[1] / 1.8 < errs[0] / 3.2, errs


def test_preconditioner_matches_dense_column_solves(oracle_mod):
    o = oracle_mod.OctOracle(_problem(3, 5, amp=0.9))
    m = o.dense_matrix()
    nc, nz = o.cells, o.problem.nz
    r = np.random.default_rng(3).uniform(-1, 1, o.n)
    e = o.apply_pinv(r)
    for c in (0, 7, nc // 2, nc - 1):
        idx = c + nc * np.arange(nz)
        block = m[np.ix_(idx, idx)]
        # the column block of A is its vertical tridiagonal part
        assert np.allclose(block, np.triu(np.tril(block, 1), -1))
        np.testing.assert_allclose(e[idx], np.linalg.solve(block, r[idx]), rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("method", ["gcr", "gmres"])
def test_solvers_match_dense_lu(oracle_mod, method):
    o = oracle_mod.OctOracle(_problem(2, 3, amp=0.6))
    m = o.dense_matrix()
    rhs = np.random.default_rng(5).uniform(-1, 1, o.n)
    ref = np.linalg.solve(m, rhs)
    x, st, log, _ = o.solve(rhs, tol=1e-12, k=8, method=method)
    assert st["status"] == oracle_mod.CONVERGED and st["detections"] == 0
    assert np.linalg.norm(x - ref) / np.linalg.norm(ref) <= 2 * np.linalg.cond(m) * 1e-12


@pytest.mark.parametrize("method", ["gcr", "gmres"])
def test_unpreconditioned_solvers_match_dense_lu(oracle_mod, method):
    o = oracle_mod.OctOracle(_problem(2, 3, amp=0.6))
    m = o.dense_matrix()
    rhs = np.random.default_rng(15).uniform(-1, 1, o.n)
    ref = np.linalg.solve(m, rhs)
    x, st, _, _ = o.solve(rhs, tol=1e-12, k=8, method=method, precond="none", max_steps=200000)
    assert st["status"] == oracle_mod.CONVERGED and st["detections"] == 0
    assert np.linalg.norm(x - ref) / np.linalg.norm(ref) <= 2 * np.linalg.cond(m) * 1e-12


def test_unpreconditioned_gcr_is_conjugate_residual(oracle_mod):
    """The O_N operator is symmetric, so with P = I every GCR(k) is the
    conjugate residual method: histories for k = 1, 2, 5 agree with a
    textbook conjugate-residual recurrence on the dense matrix while well
    above rounding."""
    o = oracle_mod.OctOracle(_problem(2, 3, amp=0.6))
    m = o.dense_matrix()
    assert np.allclose(m, m.T, rtol=0, atol=1e-13 * np.abs(m).max())
    rhs = np.random.default_rng(16).uniform(-1, 1, o.n)
    steps = 50
    hs = [o.solve(rhs, tol=1e-30, k=k, max_steps=steps, ft=False, precond="none")[3] for k in (1, 2, 5)]
    r = rhs.copy()
    p = r.copy()
    ar = m @ r
    ap = ar.copy()
    ref = []
    for _ in range(steps):
        rar = r @ ar
        alpha = rar / (ap @ ap)
        r = r - alpha * ap
        ref.append(r @ r)
        ar = m @ r
        beta = (r @ ar) / rar
        p = r + beta * p
        ap = ar + beta * ap
    ref = np.array(ref)
    keep = ref > 1e-16 * (rhs @ rhs)
    assert keep.sum() >= 20
    for h in hs:
        np.testing.assert_allclose(h[:steps][keep], ref[keep], rtol=1e-7)
    with pytest.raises(ValueError):
        o.solve(rhs, tol=1e-8, k=3, precond="diagonal")


def test_detected_fault_recovers_fault_free_run(oracle_mod):
    from paper_2103_07210_amd.inputs import FaultEvent
    o = oracle_mod.OctOracle(_problem(8, 6))
    rhs = np.random.default_rng(6).uniform(-1, 1, o.n)
    xc, sc, _, _ = o.solve(rhs, tol=1e-10, k=4)
    x, st, log, _ = o.solve(rhs, tol=1e-10, k=4, plan=[FaultEvent(6, "r", 62, idx=np.array([1000]))])
    assert [(d["step"], d["nu"]) for d in log] == [(6, 1)] and st["steps_wasted"] == 2
    assert np.array_equal(x, xc) and st["steps_executed"] == sc["steps_executed"] + 2


def _continuum(amp):
    """-div(c grad phi) on the shallow unit-sphere shell, the hill
    coefficient c of the workloads, phi = (cos(lat) cos(lon) + 3 sin(lat)^2
    - 1) cos(pi zeta), differentiated symbolically."""
    import sympy as sp
    lam, th, ze = sp.symbols("lam th ze", real=True)
    hl, ht = math.pi / 2, math.pi / 6
    hav = sp.sin((th - ht) / 2) ** 2 + sp.cos(th) * math.cos(ht) * sp.sin((lam - hl) / 2) ** 2
    c = 1 + amp * sp.exp(-(2 * sp.asin(sp.sqrt(hav)) / 0.35) ** 2) * sp.exp(-ze / 0.3)
    phi = (sp.cos(th) * sp.cos(lam) + 3 * sp.sin(th) ** 2 - 1) * sp.cos(sp.pi * ze)
    div = (sp.diff(c / sp.cos(th) * sp.diff(phi, lam), lam) / sp.cos(th)
           + sp.diff(c * sp.cos(th) * sp.diff(phi, th), th) / sp.cos(th) + sp.diff(c * sp.diff(phi, ze), ze))
    return sp.lambdify((lam, th, ze), phi, "numpy"), sp.lambdify((lam, th, ze), -div, "numpy")


def test_variable_coefficient_consistency(oracle_mod):
    """With the hill coefficient (c at the face centres): A0 phi / (control
    volume) -> -div(c grad phi) under refinement of both N and nz; a
    coefficient taken at the points instead of the faces, or a wrong control
    area, stalls the error."""
    f_phi, f_L = _continuum(0.5)
    errs = []
    for N, nz in ((8, 4), (16, 8), (32, 16)):
        o = oracle_mod.OctOracle(_problem(N, nz, amp=0.5, helmholtz=1e-300))
        lon, lat, area, _ = o.mesh()
        zeta = (np.arange(nz) + 0.5) / nz
        LON, LAT = np.tile(lon, nz), np.tile(lat, nz)
        Z = np.repeat(zeta, o.cells)
        disc = o.apply_A(f_phi(LON, LAT, Z)) / (np.tile(area, nz) / nz)
        exact = f_L(LON, LAT, Z)
        mask = np.abs(LAT) <= math.pi / 3
        errs.append(np.max(np.abs(disc - exact)[mask]) / np.max(np.abs(exact)[mask]))
    assert errs[2] < 5e-3, errs
    assert errs[0] / errs[1] > 2.5 and errs[1] / errs[2] > 2.5, errs
