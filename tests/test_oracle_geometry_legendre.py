"""Pins of the oracle's HEALPix geometry and Legendre functions (CPU only).

Geometry: the published HEALPix ring definition (Gorski et al. 2005).
Legendre: closed forms of Y_lm at low l (sympy), an arbitrary-precision library
routine at high l (mpmath), the addition theorem and Gauss-Legendre
orthonormality.
"""
import math

import mpmath
import numpy as np
import pytest
import sympy

from oracle import healpix, legendre


# ----------------------------------------------------------------- I1 geometry
@pytest.mark.parametrize("nside", [1, 2, 4, 8, 16, 64])
def test_ring_geometry_invariants(nside):
    g = healpix.ring_info(nside)
    nr = 4 * nside - 1
    assert len(g["z"]) == nr
    assert g["nphi"].sum() == 12 * nside * nside
    # rings tile the pixel index range in order
    assert g["start"][0] == 0
    assert np.all(g["start"][1:] == g["start"][:-1] + g["nphi"][:-1])
    # north/south mirror symmetry
    assert np.array_equal(g["z"][::-1], -g["z"])
    assert np.array_equal(g["nphi"][::-1], g["nphi"])
    assert np.allclose(g["phi0"][::-1], g["phi0"], rtol=0, atol=0)
    # z decreases monotonically from the north pole
    assert np.all(np.diff(g["z"]) < 0)
    # polar caps hold 2 Nside (Nside - 1) pixels each
    assert g["start"][nside - 1] == 2 * nside * (nside - 1)


def test_ring_geometry_nside1_values():
    g = healpix.ring_info(1)
    assert np.allclose(g["z"], [2.0 / 3.0, 0.0, -2.0 / 3.0], rtol=0, atol=1e-16)
    assert list(g["nphi"]) == [4, 4, 4]
    assert np.allclose(g["phi0"], [np.pi / 4, 0.0, np.pi / 4], rtol=0, atol=1e-16)


@pytest.mark.parametrize("nside", [1, 2, 8, 32])
def test_equal_area_ring_latitudes(nside):
    """Equal-area property: the spherical cap above a ring centre holds exactly
    the pixels of the rings above it plus half of the ring itself."""
    g = healpix.ring_info(nside)
    npix = 12 * nside * nside
    above = g["start"] + g["nphi"] / 2.0
    assert np.allclose(above, (1.0 - g["z"]) / 2.0 * npix, rtol=0, atol=1e-9)


# ----------------------------------------------------------------- Legendre closed forms
def _ylm_sympy(l, m):
    th, ph = sympy.symbols("theta phi", real=True)
    expr = sympy.Ynm(l, m, th, ph).expand(func=True)
    expr = sympy.simplify(expr * sympy.exp(-sympy.I * m * ph))  # lambda_lm(cos theta)
    return sympy.lambdify(th, expr, "numpy")


@pytest.mark.parametrize("nside", [1, 4, 16])
def test_lambda_closed_forms_low_l(nside):
    """I2: lambda_lm(z) equals sympy's Y_lm (Condon-Shortley) for l <= 4 at every ring."""
    z = healpix.ring_info(nside)["z"]
    lam = legendre.lambda_all(4, z)
    theta = np.arccos(z)
    for l in range(5):
        for m in range(l + 1):
            ref = np.real(np.asarray(_ylm_sympy(l, m)(theta), dtype=np.complex128))
            ref = np.broadcast_to(ref, z.shape)
            got = lam[legendre.alm_index(4, l, m)]
            assert np.allclose(got, ref, rtol=0, atol=1e-14), (l, m)


def test_lambda_textbook_values():
    """Hand-written textbook forms (independent of sympy) for l <= 2."""
    z = np.linspace(-0.95, 0.95, 13)
    s = np.sqrt(1 - z * z)
    pi = np.pi
    want = {
        (0, 0): np.full_like(z, 0.5 / np.sqrt(pi)),
        (1, 0): np.sqrt(3 / (4 * pi)) * z,
        (1, 1): -np.sqrt(3 / (8 * pi)) * s,
        (2, 0): np.sqrt(5 / (16 * pi)) * (3 * z * z - 1),
        (2, 1): -np.sqrt(15 / (8 * pi)) * s * z,
        (2, 2): np.sqrt(15 / (32 * pi)) * s * s,
    }
    lam = legendre.lambda_all(2, z)
    for (l, m), ref in want.items():
        assert np.allclose(lam[legendre.alm_index(2, l, m)], ref, rtol=0, atol=1e-15)


def _mp_lambda(l, m, z, dps):
    with mpmath.workdps(dps):
        v = mpmath.spherharm(l, m, mpmath.acos(mpmath.mpf(z)), 0)
        return mpmath.re(v)


def test_lambda_vs_mpmath_high_l():
    """I3: lambda_lm against mpmath's spherharm at high l, including rings near
    the pole (exponent rescaling) -- tolerance 1e-12 * sqrt((2l+1)/(4 pi))."""
    rs = np.random.default_rng(1234)
    cases = []
    z_ring = healpix.ring_info(1024)["z"]
    for _ in range(120):
        l = int(rs.integers(0, 2049))
        m = int(rs.integers(0, l + 1))
        z = float(z_ring[rs.integers(0, len(z_ring))])
        cases.append((l, m, z))
    # near-pole, large-m cases where the sectoral seed underflows double precision
    for (l, m) in [(2048, 30), (2048, 200), (2048, 600), (1500, 400), (2048, 2048),
                   (1024, 100), (2000, 1000)]:
        for z in (float(z_ring[0]), float(z_ring[3]), float(z_ring[20]), float(z_ring[100])):
            cases.append((l, m, z))
    by_m = {}
    for (l, m, z) in cases:
        by_m.setdefault((m, z), []).append(l)
    for (m, z), ls in by_m.items():
        lam = legendre.lambda_m(max(ls), m, np.array([z]))[:, 0]
        for l in ls:
            ref50 = _mp_lambda(l, m, z, 50)
            ref80 = _mp_lambda(l, m, z, 80)
            assert abs(ref50 - ref80) <= 1e-30 * max(1.0, abs(ref80))   # reference is stable
            tol = 1e-12 * math.sqrt((2 * l + 1) / (4 * math.pi))
            assert abs(lam[l - m] - float(ref80)) <= tol, (l, m, z, lam[l - m], ref80)


def test_lambda_vs_mpmath_pole_m0():
    """Forward recurrence on the pole-most Nside-1024 ring for m <= 2: the error
    grows with l (see the polar addition-theorem test); bound 2e-11 relative."""
    z = float(healpix.ring_info(1024)["z"][0])
    for m in range(3):
        lam = legendre.lambda_m(2048, m, np.array([z]))[:, 0]
        for l in (m + 10, 512, 1386, 2048):
            ref = float(_mp_lambda(l, m, z, 60))
            assert abs(lam[l - m] - ref) <= 2e-11 * abs(ref), (l, m)


@pytest.mark.parametrize("nside,lmax", [(4, 8), (16, 32), (64, 128)])
def test_addition_theorem(nside, lmax):
    """I4: lambda_l0^2 + 2 sum_{m>=1} lambda_lm^2 = (2l+1)/(4 pi) at every ring z."""
    z = healpix.ring_info(nside)["z"]
    lam = legendre.lambda_all(lmax, z)
    for l in range(lmax + 1):
        tot = lam[legendre.alm_index(lmax, l, 0)] ** 2
        for m in range(1, l + 1):
            tot = tot + 2 * lam[legendre.alm_index(lmax, l, m)] ** 2
        assert np.allclose(tot, (2 * l + 1) / (4 * np.pi), rtol=1e-12, atol=0)


def test_addition_theorem_polar_high_l():
    """I4 at Nside-1024 polar rings up to l = 2048 (exponent-rescaled region).

    Near z = 1 the two solutions of the l-recurrence nearly coincide, so the
    forward recurrence loses accuracy roughly like l^2 * eps (measured against
    mpmath: ~8e-12 relative at l = 2048 on the pole-most ring). The bound is
    therefore 1e-11 here and 1e-12 away from the poles."""
    z = healpix.ring_info(1024)["z"][[0, 1, 5, 50, 500, 2047]]
    lmax = 2048
    seeds = legendre.sectoral(lmax, z)
    tot = np.zeros((lmax + 1, z.size))
    for m in range(lmax + 1):
        lam = legendre.lambda_m(lmax, m, z, seeds)
        tot[m:] += (1.0 if m == 0 else 2.0) * lam ** 2
    l = np.arange(lmax + 1)[:, None]
    rel = np.abs(tot / ((2 * l + 1) / (4 * np.pi)) - 1.0)
    assert rel[:, :3].max() < 1e-11
    assert rel[:, 3:].max() < 1e-12


@pytest.mark.parametrize("lmax", [10, 64])
def test_gauss_legendre_orthonormality(lmax):
    """I4: 2 pi sum_j w_j lambda_lm(x_j) lambda_l'm(x_j) = delta_ll' on Gauss nodes."""
    x, w = np.polynomial.legendre.leggauss(lmax + 2)
    lam = legendre.lambda_all(lmax, x)
    for m in range(0, lmax + 1, max(1, lmax // 8)):
        i0 = legendre.alm_index(lmax, m, m)
        L = lam[i0:i0 + lmax - m + 1]
        G = 2 * np.pi * (L * w) @ L.T
        assert np.allclose(G, np.eye(lmax - m + 1), rtol=0, atol=1e-12)


def test_parity_symmetry():
    """lambda_lm(-z) = (-1)^(l+m) lambda_lm(z), and lambda_lm(0) = 0 for l+m odd."""
    lmax = 40
    z = np.array([0.0, 0.3, -0.3, 0.9, -0.9])
    lam = legendre.lambda_all(lmax, z)
    for m in range(lmax + 1):
        for l in range(m, lmax + 1):
            row = lam[legendre.alm_index(lmax, l, m)]
            sgn = (-1) ** (l + m)
            assert abs(row[2] - sgn * row[1]) <= 1e-14 * max(1, abs(row[1]))
            assert abs(row[4] - sgn * row[3]) <= 1e-14 * max(1, abs(row[3]))
            if (l + m) % 2:
                assert row[0] == 0.0
