"""Pins of the oracle's operator A, hill coefficient and column preconditioner
against facts fixed by mathematics, independently of the oracle's own code.

Operator (stand-in for the elliptic operator L of the paper's Eq. (1)):
A = A0 + sigma diag(A0), A0 = -V div(c grad) in flux form on the unit-sphere
shallow shell, periodic in longitude, zero flux through poles, bottom and top.
Preconditioner: P = vertical tridiagonal part of A (the paper only says GCR is
left-preconditioned for the domain anisotropy, Section 2).
"""
import math

import numpy as np
import pytest
import sympy as sp

from paper_2103_07210_amd.inputs import Problem


def _centres(pb):
    lon = (np.arange(pb.nx) + 0.5) * 2 * np.pi / pb.nx
    lat = -np.pi / 2 + (np.arange(pb.ny) + 0.5) * np.pi / pb.ny
    zeta = (np.arange(pb.nz) + 0.5) / pb.nz
    Z, LAT, LON = np.meshgrid(zeta, lat, lon, indexing="ij")
    return LON, LAT, Z


def test_hill_matches_chord_length_distance(oracle_mod):
    """Great-circle distance from the chord between unit vectors (an
    independent formula from the haversine used by the oracle)."""
    pb = Problem(8, 4, 2)
    o = oracle_mod.Oracle(pb)
    rng = np.random.default_rng(7)
    for _ in range(200):
        lon = rng.uniform(0, 2 * np.pi)
        lat = rng.uniform(-np.pi / 2, np.pi / 2)
        u = np.array([np.cos(lat) * np.cos(lon), np.cos(lat) * np.sin(lon), np.sin(lat)])
        v = np.array([np.cos(pb.hill_lat) * np.cos(pb.hill_lon),
                      np.cos(pb.hill_lat) * np.sin(pb.hill_lon), np.sin(pb.hill_lat)])
        gc = 2 * np.arcsin(min(1.0, np.linalg.norm(u - v) / 2))
        assert o.hill(lon, lat) == pytest.approx(np.exp(-(gc / pb.hill_width) ** 2), rel=1e-12, abs=1e-300)
    # exactly 1 at the centre, and tiny at the antipode
    assert o.hill(pb.hill_lon, pb.hill_lat) == 1.0
    assert o.hill(pb.hill_lon + np.pi, -pb.hill_lat) < 1e-30


def test_shift_is_relative_to_diagonal(oracle_mod):
    """A0 has the constants as null space, so A 1 = sigma D0 = sigma/(1+sigma)
    diag(A) -- with diag(A) read off the assembled matrix."""
    pb = Problem(6, 5, 4, hill_amp=0.8)
    o = oracle_mod.Oracle(pb)
    dense = o.dense_matrix()
    a1 = dense @ np.ones(pb.n)
    sig = pb.helmholtz
    np.testing.assert_allclose(a1, sig / (1 + sig) * np.diag(dense), rtol=1e-11, atol=1e-15)
    o0 = oracle_mod.Oracle(Problem(6, 5, 4, hill_amp=0.8, helmholtz=0.0))
    y = o0.apply_A(np.ones(pb.n))
    assert np.max(np.abs(y)) < 1e-14 * np.max(np.abs(np.diag(o0.dense_matrix())))


@pytest.mark.parametrize("shape", [(6, 4, 3), (5, 6, 4)])
def test_symmetric_positive_definite(oracle_mod, shape):
    pb = Problem(*shape, hill_amp=0.9, hill_lat=0.3)
    o = oracle_mod.Oracle(pb)
    m = o.dense_matrix()
    np.testing.assert_allclose(m, m.T, rtol=0, atol=1e-15 * np.abs(m).max())
    ev = np.linalg.eigvalsh(0.5 * (m + m.T))
    # Gershgorin: each row has diag (1+s) D0 and off-diagonal mass D0.
    d = np.diag(m)
    assert ev.min() >= 0.999 * np.min(d * pb.helmholtz / (1 + pb.helmholtz))
    # exactly 7-point: at most 7 non-zeros per row
    assert np.max(np.count_nonzero(m, axis=1)) <= 7


def _continuum_operator(pb):
    """-div(c grad phi) on the shallow unit-sphere shell for
    phi = (cos(lat) cos(lon) + 3 sin(lat)^2 - 1) cos(pi zeta), with the hill
    coefficient c, differentiated symbolically."""
    lam, th, ze = sp.symbols("lam th ze", real=True)
    H = sp.Float(pb.shell_depth)
    hav = sp.sin((th - pb.hill_lat) / 2) ** 2 + sp.cos(th) * sp.cos(pb.hill_lat) * sp.sin((lam - pb.hill_lon) / 2) ** 2
    gc = 2 * sp.asin(sp.sqrt(hav))
    c = 1 + pb.hill_amp * sp.exp(-(gc / pb.hill_width) ** 2) * sp.exp(-ze / pb.decay_z)
    phi = (sp.cos(th) * sp.cos(lam) + 3 * sp.sin(th) ** 2 - 1) * sp.cos(sp.pi * ze)
    # z = H zeta, so d/dz = (1/H) d/dzeta
    div = (sp.diff(c / sp.cos(th) * sp.diff(phi, lam), lam) / sp.cos(th)
           + sp.diff(c * sp.cos(th) * sp.diff(phi, th), th) / sp.cos(th)
           + sp.diff(c * sp.diff(phi, ze) / H, ze) / H)
    f_phi = sp.lambdify((lam, th, ze), phi, "numpy")
    f_L = sp.lambdify((lam, th, ze), -div, "numpy")
    return f_phi, f_L


def _consistency_error(oracle_mod, pb, f_phi, f_L):
    o = oracle_mod.Oracle(pb)
    LON, LAT, Z = _centres(pb)
    phi = f_phi(LON, LAT, Z)
    vol = np.cos(LAT) * (2 * np.pi / pb.nx) * (np.pi / pb.ny) * (pb.shell_depth / pb.nz)
    disc = o.apply_A(phi) / vol
    exact = f_L(LON, LAT, Z)
    mask = np.abs(LAT) <= np.pi / 3
    return np.max(np.abs(disc - exact)[mask]) / np.max(np.abs(exact)[mask])


@pytest.mark.parametrize("amp", [0.0, 0.5])
def test_second_order_consistency_against_closed_form(oracle_mod, amp):
    """(A0 phi)_c / V_c -> -div(c grad phi) at second order on |lat| <= 60 deg.
    With amp = 0 the exact value is (l(l+1) + (pi/H)^2) phi (spherical
    harmonics of degree 1 and 2 times cos(pi zeta)); with the hill the
    reference is a symbolic derivative.  A coefficient evaluated at a cell
    centre instead of a face centre, a wrong metric factor or a wrong face
    area breaks the factor-4 error reduction."""
    base = Problem(32, 16, 8, hill_amp=amp, helmholtz=0.0)
    f_phi, f_L = _continuum_operator(base)
    errs = []
    for m in (1, 2, 4):
        pb = Problem(32 * m, 16 * m, 8 * m, hill_amp=amp, helmholtz=0.0)
        errs.append(_consistency_error(oracle_mod, pb, f_phi, f_L))
    assert errs[2] < 0.05
    assert errs[0] / errs[1] > 3.3 and errs[1] / errs[2] > 3.5, errs
    if amp == 0.0:
        # cross-check the symbolic reference with the eigenvalue closed form
        LON, LAT, Z = _centres(Problem(8, 6, 4))
        y1 = np.cos(LAT) * np.cos(LON)
        y2 = 3 * np.sin(LAT) ** 2 - 1
        k2 = np.pi ** 2
        closed = ((2 + k2) * y1 + (6 + k2) * y2) * np.cos(np.pi * Z)
        np.testing.assert_allclose(f_L(LON, LAT, Z), closed, rtol=1e-10, atol=1e-10)


def test_pinv_solves_vertical_blocks_of_assembled_operator(oracle_mod):
    """P^{-1} r equals a dense solve with the vertical tridiagonal blocks of
    the assembled A (diagonal and the level-to-level couplings)."""
    pb = Problem(5, 4, 7, hill_amp=0.7)
    o = oracle_mod.Oracle(pb)
    m = o.dense_matrix()
    r = np.random.default_rng(3).uniform(-1, 1, pb.n)
    e = o.apply_pinv(r).reshape(-1)
    plane = pb.nx * pb.ny
    for j in range(pb.ny):
        for i in range(pb.nx):
            ids = i + pb.nx * j + plane * np.arange(pb.nz)
            blk = m[np.ix_(ids, ids)]
            tri = np.triu(np.tril(blk, 1), -1)
            np.testing.assert_array_equal(blk, tri)  # only vertical neighbours couple in a column
            ref = np.linalg.solve(tri, r[ids])
            np.testing.assert_allclose(e[ids], ref, rtol=1e-13, atol=1e-15)
    assert np.all(np.isfinite(e))


def test_pinv_single_level_is_jacobi(oracle_mod):
    pb = Problem(7, 3, 1, hill_amp=0.4)
    o = oracle_mod.Oracle(pb)
    r = np.random.default_rng(5).uniform(-1, 1, pb.n)
    d = np.diag(o.dense_matrix())
    np.testing.assert_allclose(o.apply_pinv(r).reshape(-1), r / d, rtol=1e-15)


def test_dot_left_to_right(oracle_mod):
    o = oracle_mod.Oracle(Problem(4, 2, 2))
    a = np.array([1e16, 1.0, -1e16, 1.0] * 4)
    b = np.ones(16)
    acc = 0.0
    for v in a:  # the sequential sum loses the +1 that follows each 1e16
        acc += v
    assert o.dot(a, b) == acc
    assert acc != math.fsum(a)
