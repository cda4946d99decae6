"""Pins of the oracle's ring sums and spherical-harmonic transform pair (CPU only).

Brute-force term-by-term sums on tiny inputs, the exact adjointness of the
pixel-area analysis and the synthesis, the exact rotation / mirror symmetries
of HEALPix rings, and closed-form single-mode synthesis.
"""
import numpy as np
import pytest
import sympy

from oracle import healpix, sht
from oracle.legendre import alm_index, n_alm


def _rand_alm(lmax, rs, real_m0=True):
    a = rs.standard_normal(n_alm(lmax)) + 1j * rs.standard_normal(n_alm(lmax))
    if real_m0:
        a[:lmax + 1] = a[:lmax + 1].real
    return a


@pytest.mark.parametrize("nside,lmax", [(1, 3), (2, 5), (4, 8), (4, 15), (8, 16), (8, 31), (16, 33), (16, 63)])
def test_ring_sums_match_direct(nside, lmax):
    """FFT + bin folding equals the term-by-term sums, aliasing included (lmax up to
    4 nside - 1: every polar ring folds several frequencies into each bin)."""
    rs = np.random.default_rng(nside * 100 + lmax)
    f = rs.standard_normal(healpix.npix(nside))
    G = sht.ring_analysis(f, nside, lmax)
    Gd = sht.ring_analysis_direct(f, nside, lmax)
    assert np.allclose(G, Gd, rtol=0, atol=1e-12 * np.abs(Gd).max())
    F = rs.standard_normal(G.shape) + 1j * rs.standard_normal(G.shape)
    F[:, 0] = F[:, 0].real
    x = sht.ring_synthesis(F, nside, lmax)
    xd = sht.ring_synthesis_direct(F, nside, lmax)
    assert np.allclose(x, xd, rtol=0, atol=1e-12 * np.abs(xd).max())


@pytest.mark.parametrize("nside,lmax", [(2, 4), (4, 8), (8, 16), (16, 32), (8, 31)])
def test_adjointness(nside, lmax):
    """I5: Omega <f, alm2map(a)>_pix = <a, map2alm(f)>_alm (exact identity)."""
    rs = np.random.default_rng(7 + nside + lmax)
    f = rs.standard_normal(healpix.npix(nside))
    a = _rand_alm(lmax, rs)
    lhs = healpix.pixel_area(nside) * float(np.dot(f, sht.alm2map(a, nside, lmax)))
    rhs = sht.alm_dot(a, sht.map2alm(f, nside, lmax), lmax)
    assert abs(lhs - rhs) <= 1e-13 * max(abs(lhs), 1e-300) * 10 + 1e-14


@pytest.mark.parametrize("nside,lmax", [(4, 8), (8, 16), (16, 32)])
def test_quarter_turn_and_mirror(nside, lmax):
    """I6: rolling every ring by n_phi/4 multiplies a_lm by exp(-i m pi/2);
    swapping ring i with ring 4 Nside - i multiplies a_lm by (-1)^(l+m)."""
    rs = np.random.default_rng(11 + nside)
    f = rs.standard_normal(healpix.npix(nside))
    g = healpix.ring_info(nside)
    a = sht.map2alm(f, nside, lmax)
    ell = sht.alm_ell(lmax)
    em = np.concatenate([np.full(lmax + 1 - m, m) for m in range(lmax + 1)])
    rolled = np.empty_like(f)
    mirrored = np.empty_like(f)
    nr = len(g["z"])
    for r in range(nr):
        s, n = g["start"][r], g["nphi"][r]
        rolled[s:s + n] = np.roll(f[s:s + n], n // 4)
        r2 = nr - 1 - r
        s2 = g["start"][r2]
        mirrored[s:s + n] = f[s2:s2 + n]
    a_rot = sht.map2alm(rolled, nside, lmax)
    assert np.allclose(a_rot, a * np.exp(-1j * em * np.pi / 2), rtol=0, atol=1e-13 * np.abs(a).max())
    a_mir = sht.map2alm(mirrored, nside, lmax)
    assert np.allclose(a_mir, a * (-1.0) ** (ell + em), rtol=0, atol=1e-13 * np.abs(a).max())


def test_single_mode_synthesis_closed_form():
    """I7: alm2map of a single (l, m) equals the closed-form Y_lm (sympy) at every
    pixel: a_lm = 1 gives 2 Re Y_lm (m > 0) or Y_l0; a_lm = i gives -2 Im Y_lm."""
    nside, lmax = 4, 4
    theta, phi = healpix.pixel_angles(nside)
    th, ph = sympy.symbols("theta phi", real=True)
    for l in range(lmax + 1):
        for m in range(l + 1):
            y = sympy.lambdify((th, ph), sympy.Ynm(l, m, th, ph).expand(func=True), "numpy")
            yv = np.asarray(y(theta, phi), dtype=np.complex128) * np.ones_like(theta)
            a = np.zeros(n_alm(lmax), dtype=np.complex128)
            a[alm_index(lmax, l, m)] = 1.0
            got = sht.alm2map(a, nside, lmax)
            want = yv.real if m == 0 else 2 * yv.real
            assert np.allclose(got, want, rtol=0, atol=1e-14), (l, m)
            if m > 0:
                a[alm_index(lmax, l, m)] = 1j
                got = sht.alm2map(a, nside, lmax)
                assert np.allclose(got, -2 * yv.imag, rtol=0, atol=1e-14), (l, m)


def test_monopole_exact():
    """The pixel-area analysis of a constant map is exact for the monopole:
    a_00 = Omega * npix * c / sqrt(4 pi) = sqrt(4 pi) c."""
    nside, lmax = 8, 16
    c = 2.5
    a = sht.map2alm(np.full(healpix.npix(nside), c), nside, lmax)
    assert abs(a[0] - np.sqrt(4 * np.pi) * c) < 1e-13


def test_analysis_inverts_synthesis_approximately():
    """Omega Y^dagger Y is close to (not equal to) the identity at lmax <= Nside."""
    nside, lmax = 16, 16
    rs = np.random.default_rng(3)
    a = _rand_alm(lmax, rs)
    back = sht.map2alm(sht.alm2map(a, nside, lmax), nside, lmax)
    rel = np.linalg.norm(back - a) / np.linalg.norm(a)
    assert 1e-6 < rel < 0.05


def test_column_analysis_closed_form():
    """map2alm_columns (used for spot checks of large transforms) against the
    definition written with closed-form Y_lm (sympy), l <= 4: a_lm = Omega sum_p
    conj(Y_lm(theta_p, phi_p)) f_p."""
    nside, lmax = 4, 4
    theta, phi = healpix.pixel_angles(nside)
    f = np.random.default_rng(11).standard_normal(theta.size)
    cols = sht.map2alm_columns(f, nside, lmax, [0, 1, 2, 4])
    th, ph = sympy.symbols("theta phi", real=True)
    omega = 4 * np.pi / theta.size
    for m, got in cols.items():
        for l in range(m, lmax + 1):
            y = sympy.lambdify((th, ph), sympy.Ynm(l, m, th, ph).expand(func=True), "numpy")
            yv = np.asarray(y(theta, phi), dtype=np.complex128) * np.ones_like(theta)
            want = omega * np.sum(np.conj(yv) * f)
            assert abs(got[l - m] - want) < 1e-13, (l, m)


def test_column_transforms_match_full_transforms():
    """The column-restricted pair equals the full pair on the same columns, and
    keeps the exact adjointness: Omega <f, Y a> = <Omega Y^dagger f, a>."""
    nside, lmax = 8, 20
    rs = np.random.default_rng(12)
    f = rs.standard_normal(healpix.npix(nside))
    ms = [0, 3, 9, 20]
    full = sht.map2alm(f, nside, lmax)
    cols = sht.map2alm_columns(f, nside, lmax, ms)
    for m in ms:
        i0 = alm_index(lmax, m, m)
        assert np.allclose(cols[m], full[i0:i0 + lmax - m + 1], rtol=0, atol=1e-13)
    a = {m: rs.standard_normal(lmax - m + 1) + 1j * rs.standard_normal(lmax - m + 1) for m in ms}
    a[0] = a[0].real
    packed = np.zeros(n_alm(lmax), dtype=np.complex128)
    for m in ms:
        i0 = alm_index(lmax, m, m)
        packed[i0:i0 + lmax - m + 1] = a[m]
    got = sht.alm2map_columns(a, nside, lmax)
    assert np.allclose(got, sht.alm2map(packed, nside, lmax), rtol=0, atol=1e-12)
    lhs = healpix.pixel_area(nside) * np.dot(f, got)
    rhs = sum((1.0 if m == 0 else 2.0) * np.sum(cols[m] * np.conj(a[m])).real for m in ms)
    assert abs(lhs - rhs) < 1e-12 * max(1.0, abs(lhs))
