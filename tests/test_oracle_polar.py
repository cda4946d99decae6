"""Pins of the polarised oracle (CPU only).

Spin-weighted functions: the Newman-Penrose eth construction of sY_lm from the
spin-0 Y_lm (sympy, l <= 4), Goldberg's explicit sum in arbitrary precision
(mpmath) up to l = 2048 including near-pole rings, the spin-2 addition theorem,
Gauss-Legendre orthonormality and the reflection symmetries. Transforms: the
defining direct sums at every pixel (aliasing included), adjointness, rotation
and mirror symmetries. The sweep: Eq. (3) with Nbar and T written out, Eq. (4)
with S and T written out, the reduction to the spin-0 filter when the fields
decouple, the full-sky uniform-noise closed form, and the dense fixed point with
its convergence rate.
"""
import math

import mpmath
import numpy as np
import pytest
import sympy

from oracle import healpix, legendre, messenger, polar, sht
from oracle.legendre import alm_index, n_alm
from paper_1211_0585_amd import synth


def _rel(x, ref):
    return float(np.linalg.norm(np.ravel(x - ref)) / max(np.linalg.norm(np.ravel(ref)), 1e-300))


# ----------------------------------------------------------------- spin-weighted functions
def _eth_functions(l, m):
    """(2)Y_lm and (-2)Y_lm without exp(i m phi), from Y_lm by two eth (eth-bar) steps:
    eth eta = -sin^s (d_theta + i/sin d_phi)(sin^-s eta), eth-bar eta = -sin^-s (d_theta -
    i/sin d_phi)(sin^s eta), sY = sqrt((l-s)!/(l+s)!) eth^s Y (s > 0), sqrt((l+s)!/(l-s)!)
    (-1)^s eth-bar^-s Y (s < 0)."""
    th, ph = sympy.symbols("theta phi", real=True)

    def eth(eta, s, sign):
        f = sympy.sin(th) ** (-sign * s)
        return -sympy.sin(th) ** (sign * s) * (sympy.diff(f * eta, th) + sign * sympy.I / sympy.sin(th)
                                               * sympy.diff(f * eta, ph))

    Y = sympy.Ynm(l, m, th, ph).expand(func=True)
    norm = sympy.sqrt(sympy.factorial(l - 2) / sympy.factorial(l + 2))
    p2 = norm * eth(eth(Y, 0, 1), 1, 1)
    m2 = norm * eth(eth(Y, 0, -1), -1, -1)
    out = []
    for e in (p2, m2):
        out.append(sympy.lambdify(th, sympy.simplify(e * sympy.exp(-sympy.I * m * ph)), "numpy"))
    return out


@pytest.mark.parametrize("l", [2, 3, 4])
def test_goldberg_equals_eth_construction(l):
    tv = np.array([0.05, 0.4, 1.1, np.pi / 2, 2.3, 3.1])
    for m in range(-l, l + 1):
        f2, fm2 = _eth_functions(l, m)
        assert np.max(np.abs(np.real(f2(tv)) - polar.goldberg(l, m, 2, tv))) < 1e-12
        assert np.max(np.abs(np.real(fm2(tv)) - polar.goldberg(l, m, -2, tv))) < 1e-12


def test_goldberg_spin0_is_condon_shortley_ylm():
    th = np.linspace(0.05, 3.09, 9)
    for l in range(7):
        for m in range(l + 1):
            ref = legendre.lambda_m(l, m, np.cos(th))[l - m]
            assert np.max(np.abs(polar.goldberg(l, m, 0, th) - ref)) < 1e-13


@pytest.mark.parametrize("s", [2, -2])
def test_recurrence_matches_goldberg_low_l(s):
    """Every ring of Nside 8 and a few angles near both poles, l <= 10."""
    z = np.concatenate([healpix.ring_info(8)["z"], np.cos([1e-3, 0.02, np.pi - 0.02, np.pi - 1e-3])])
    th = np.arccos(z)
    for m in range(11):
        vals = polar.spin_lambda_m(10, m, s, z)
        for l in range(m, 11):
            ref = polar.goldberg(l, m, s, th)
            assert np.max(np.abs(vals[l - m] - ref)) < 2e-14 * max(1.0, np.max(np.abs(ref))), (l, m)


def _goldberg_mp(l, m, s, theta):
    """Goldberg's sum in arbitrary precision (enough digits for its cancellation)."""
    with mpmath.workdps(int(0.65 * l) + 40):
        t = mpmath.mpf(theta) / 2
        sh, ch = mpmath.sin(t), mpmath.cos(t)
        pre = (-1) ** m * mpmath.sqrt(mpmath.factorial(l + m) * mpmath.factorial(l - m) * (2 * l + 1)
                                      / (4 * mpmath.pi * mpmath.factorial(l + s) * mpmath.factorial(l - s)))
        tot = mpmath.mpf(0)
        for r in range(l - s + 1):
            k = r + s - m
            if k < 0 or k > l + s:
                continue
            e = 2 * r + s - m
            tot += mpmath.binomial(l - s, r) * mpmath.binomial(l + s, k) * (-1) ** (l - r - s) * ch ** e * sh ** (
                2 * l - e)
        return float(pre * tot)


@pytest.mark.slow
def test_recurrence_matches_mpmath_high_l():
    """Random (l, m, ring) of Nside 1024 up to l = 2048 incl. the pole-most rings
    (exercises the exponent carrying) against Goldberg's sum in mpmath. Bound as for
    the spin-0 functions: the forward recurrence loses ~ l^2 eps near the poles."""
    rs = np.random.default_rng(5)
    g = healpix.ring_info(1024)
    zs = g["z"]
    cases = [(2048, 3, 0), (2048, 40, 1), (1500, 1499, 300), (2000, 2, 5), (700, 650, 2047),
             (1024, 512, 900), (300, 250, 10)]
    for _ in range(10):
        l = int(rs.integers(2, 2049))
        m = int(rs.integers(0, l + 1))
        cases.append((l, m, int(rs.integers(0, len(zs)))))
    for l, m, r in cases:
        for s in (2, -2):
            got = polar.spin_lambda_m(l, m, s, zs[r:r + 1])[l - m, 0]
            ref = _goldberg_mp(l, m, s, math.acos(zs[r]))
            tol = 1e-12 * math.sqrt((2 * l + 1) / (4 * math.pi)) * max(1.0, (l / 1000.0) ** 2 * 10)
            assert abs(got - ref) <= tol, (l, m, r, s, got, ref)


@pytest.mark.parametrize("nside,lmax", [(8, 24), (64, 180)])
def test_spin2_addition_theorem(nside, lmax):
    """sum over m = -l..l of |(2)Y_lm|^2 = (2l+1)/(4 pi) at every ring, l >= 2
    ((2)lambda_{l,-m} = (-1)^m (-2)lambda_lm turns the negative m into the s = -2 row)."""
    z = healpix.ring_info(nside)["z"]
    acc = np.zeros((lmax + 1, z.size))
    s2 = polar.spin_sectoral(lmax, 2, z)
    sm2 = polar.spin_sectoral(lmax, -2, z)
    for m in range(lmax + 1):
        p = polar.spin_lambda_m(lmax, m, 2, z, s2)
        q = polar.spin_lambda_m(lmax, m, -2, z, sm2)
        acc[m:] += p ** 2 + (q ** 2 if m > 0 else 0.0)
    l = np.arange(lmax + 1)
    ref = (2 * l + 1) / (4 * np.pi)
    assert np.max(np.abs(acc[2:] / ref[2:, None] - 1.0)) < 1e-12
    assert np.all(acc[:2] == 0.0)


@pytest.mark.parametrize("s", [2, -2])
def test_gauss_legendre_orthonormality(s):
    lmax = 40
    x, w = np.polynomial.legendre.leggauss(lmax + 4)
    for m in (0, 1, 2, 7, 33):
        v = polar.spin_lambda_m(lmax, m, s, x)
        G = 2 * np.pi * (v * w) @ v.T
        l = np.arange(m, lmax + 1)
        expect = np.diag((l >= 2).astype(float))
        assert np.max(np.abs(G - expect)) < 1e-12


def test_reflection_symmetries():
    """sY_{l,-m} = (-1)^{s+m} conj(-sY_lm) (Goldberg, negative m) and
    s_lambda_lm(-z) = (-1)^{l+m} (-s)_lambda_lm(z) (recurrence at mirrored rings)."""
    th = np.array([0.3, 1.0, 1.9])
    for l in range(2, 7):
        for m in range(0, l + 1):
            for s in (2, -2):
                assert np.allclose(polar.goldberg(l, -m, s, th), (-1) ** (s + m) * polar.goldberg(l, m, -s, th),
                                   rtol=0, atol=1e-14)
    z = healpix.ring_info(16)["z"]
    for m in (0, 1, 5, 20):
        for s in (2, -2):
            a = polar.spin_lambda_m(40, m, s, -z)
            b = polar.spin_lambda_m(40, m, -s, z)
            sign = (-1.0) ** (np.arange(m, 41) + m)
            assert np.max(np.abs(a - sign[:, None] * b)) < 1e-12


# ----------------------------------------------------------------- polarised transforms
def _rand_alm(lmax, seed):
    rs = np.random.default_rng(seed)
    a = rs.standard_normal((3, n_alm(lmax))) + 1j * rs.standard_normal((3, n_alm(lmax)))
    a[:, :lmax + 1] = a[:, :lmax + 1].real
    for f in (1, 2):                                   # no E, B modes below l = 2
        for m in range(2):
            for l in range(m, 2):
                a[f, alm_index(lmax, l, m)] = 0.0
    return a


@pytest.mark.parametrize("nside,lmax", [(1, 2), (1, 4), (2, 5), (2, 9), (4, 11)])
def test_transforms_equal_direct_sums(nside, lmax):
    """Ring sums + recurrences against the defining sums over every pixel (Goldberg
    functions, Q +/- iU = sum a_{+/-2} (+/-2)Y); lmax above 3 Nside exercises aliasing."""
    a = _rand_alm(lmax, 1)
    assert _rel(polar.alm2map(a, nside, lmax), polar.alm2map_direct(a, nside, lmax)) < 1e-13
    f = np.random.default_rng(2).standard_normal((3, 12 * nside * nside))
    assert _rel(polar.map2alm(f, nside, lmax), polar.map2alm_direct(f, nside, lmax)) < 1e-13


@pytest.mark.parametrize("nside,lmax", [(2, 7), (8, 16), (16, 40)])
def test_adjointness(nside, lmax):
    """Omega sum_p f . alm2map(a) = <a, map2alm(f)> over T, E, B."""
    a = _rand_alm(lmax, 3)
    f = np.random.default_rng(4).standard_normal((3, 12 * nside * nside))
    lhs = healpix.pixel_area(nside) * np.sum(f * polar.alm2map(a, nside, lmax))
    rhs = polar.alm_dot(a, polar.map2alm(f, nside, lmax), lmax)
    assert abs(lhs - rhs) <= 1e-13 * (abs(lhs) + 1.0)


def test_temperature_channel_is_spin0_transform():
    nside, lmax = 8, 16
    a = _rand_alm(lmax, 5)
    assert np.array_equal(polar.alm2map(a, nside, lmax)[0], sht.alm2map(a[0], nside, lmax))
    b = a.copy()
    b[1:] = 0.0
    out = polar.alm2map(b, nside, lmax)
    assert np.all(out[1:] == 0.0)


def test_quarter_turn_rotation():
    """Rolling every ring by n_phi / 4 pixels multiplies a_lm by exp(-i m pi/2) for
    T, E and B alike (rotations about the pole keep the local polarisation frame)."""
    nside, lmax = 8, 20
    f = np.random.default_rng(6).standard_normal((3, 12 * nside * nside))
    g = healpix.ring_info(nside)
    rot = np.empty_like(f)
    for s, n in zip(g["start"], g["nphi"]):
        rot[:, s:s + n] = np.roll(f[:, s:s + n], n // 4, axis=1)
    a = polar.map2alm(f, nside, lmax)
    b = polar.map2alm(rot, nside, lmax)
    m = np.concatenate([np.full(lmax + 1 - mm, mm) for mm in range(lmax + 1)])
    assert _rel(b, a * np.exp(-1j * m * np.pi / 2)[None]) < 1e-13


def test_mirror_symmetry():
    """Ring i <-> 4 Nside - i with U -> -U maps (T, E, B) to (-1)^{l+m} (T, E, -B)."""
    nside, lmax = 8, 20
    f = np.random.default_rng(7).standard_normal((3, 12 * nside * nside))
    g = healpix.ring_info(nside)
    mir = np.empty_like(f)
    nr = len(g["z"])
    for r in range(nr):
        s, n = g["start"][r], g["nphi"][r]
        s2 = g["start"][nr - 1 - r]
        mir[:, s:s + n] = f[:, s2:s2 + n]
    mir[2] *= -1.0
    a = polar.map2alm(f, nside, lmax)
    b = polar.map2alm(mir, nside, lmax)
    ell = sht.alm_ell(lmax)
    m = np.concatenate([np.full(lmax + 1 - mm, mm) for mm in range(lmax + 1)])
    sign = (-1.0) ** (ell + m)
    expect = np.stack([sign * a[0], sign * a[1], -sign * a[2]])
    assert _rel(b, expect) < 1e-13


# ----------------------------------------------------------------- Eq. (3), Eq. (4), tau
def _spd_ninv(npx, seed):
    rs = np.random.default_rng(seed)
    A = rs.standard_normal((npx, 3, 3))
    N = A @ np.transpose(A, (0, 2, 1)) + 0.3 * np.eye(3)
    Ninv = np.linalg.inv(N)
    return np.stack([Ninv[:, 0, 0], Ninv[:, 1, 1], Ninv[:, 2, 2], Ninv[:, 0, 1], Ninv[:, 0, 2], Ninv[:, 1, 2]]), N


def test_tau_is_smallest_noise_eigenvalue():
    n6, N = _spd_ninv(50, 1)
    M = polar.ninv_matrices(n6)
    tau = polar.tau_of(M)
    assert abs(tau - np.linalg.eigvalsh(N)[:, 0].min()) <= 1e-12 * tau
    # N - tau 1 is positive semi-definite at every pixel, singular at one
    ev = np.linalg.eigvalsh(N - tau * np.eye(3))
    assert ev.min() > -1e-12 and abs(ev[:, 0].min()) < 1e-12
    # diagonal N: the paper's min(diag N)
    d6 = np.zeros_like(n6)
    d6[:3] = n6[:3]
    assert polar.tau_of(polar.ninv_matrices(d6)) == 1.0 / d6[:3].max()


@pytest.mark.parametrize("lam", [1.0, 3.7, 1e4])
def test_pixel_update_is_eq3(lam):
    """(Nbar^-1 + (lambda T)^-1) t = Nbar^-1 d + (lambda T)^-1 s, Nbar = N - tau 1, solved
    directly at every pixel where Nbar is invertible."""
    n6, N = _spd_ninv(40, 2)
    M = polar.ninv_matrices(n6)
    tau = polar.tau_of(M)
    rs = np.random.default_rng(3)
    s, d = rs.standard_normal((2, 3, 40))
    t = polar.pixel_update(s, d, M, lam, tau)
    for p in range(40):
        Nbar = N[p] - tau * np.eye(3)
        if np.linalg.eigvalsh(Nbar)[0] < 1e-6:
            continue
        Ni = np.linalg.inv(Nbar)
        ref = np.linalg.solve(Ni + np.eye(3) / (lam * tau), Ni @ d[:, p] + s[:, p] / (lam * tau))
        assert np.max(np.abs(t[:, p] - ref)) < 1e-10 * (1 + np.max(np.abs(ref)))


def test_pixel_update_diagonal_reduces_to_spin0_weight_and_masks():
    rs = np.random.default_rng(4)
    npx = 64
    n6 = np.zeros((6, npx))
    n6[:3] = rs.uniform(0.1, 2.0, (3, npx))
    mask = rs.integers(0, 4, npx).astype(np.uint8)
    M = polar.ninv_matrices(n6, mask)
    tau = polar.tau_of(M)
    s, d = rs.standard_normal((2, 3, npx))
    t = polar.pixel_update(s, d, M, 7.5, tau)
    for f in range(3):
        q = M[:, f, f]
        w = messenger.pixel_weight(q, 7.5, tau)
        assert np.allclose(t[f], s[f] + w * (d[f] - s[f]), rtol=1e-14, atol=1e-14)
    # unobserved components keep s exactly
    assert np.array_equal(t[0][(mask & 1) == 0], s[0][(mask & 1) == 0])
    assert np.array_equal(t[1][(mask & 2) == 0], s[1][(mask & 2) == 0])


@pytest.mark.parametrize("lam", [1.0, 40.0])
def test_filter_is_eq4(lam):
    """(S^-1 + (lambda T)^-1) s = (lambda T)^-1 a with T = tau Omega 1, for l >= 2 where
    the 3x3 C_l is invertible; symmetric, eigenvalues in [0, 1)."""
    lmax = 30
    cl4 = synth.cl_pol(synth.cl_power_law(lmax))
    tau, omega = 2.3, 0.01
    F = polar.harmonic_filter(cl4, lam, tau, omega)
    C = polar.cl_matrices(cl4)
    mu = lam * tau * omega
    for l in range(2, lmax + 1):
        ref = np.linalg.solve(np.linalg.inv(C[l]) + np.eye(3) / mu, np.eye(3) / mu)
        assert np.max(np.abs(F[l] - ref)) < 1e-13
        assert np.max(np.abs(F[l] - F[l].T)) < 1e-14
        ev = np.linalg.eigvalsh(F[l])
        assert ev.min() >= 0 and ev.max() < 1
    assert np.all(F[:2, 1:] == 0) and np.all(F[:2, :, 1:] == 0)


def test_filter_without_polarisation_is_spin0_filter():
    lmax = 20
    cl = synth.cl_power_law(lmax)
    cl4 = np.stack([cl, 0 * cl, 0 * cl, 0 * cl])
    F = polar.harmonic_filter(cl4, 5.0, 0.7, 0.02)
    assert np.allclose(F[:, 0, 0], messenger.harmonic_filter(cl, 5.0, 0.7, 0.02), rtol=1e-14, atol=0)
    assert np.all(F[:, 1:, 1:] == 0)


# ----------------------------------------------------------------- the iteration
def test_decoupled_temperature_equals_spin0_solve():
    """TE = 0 and no T-P noise correlation: the T map of the polarised solve is the
    spin-0 solve of T with N^-1_TT (up to rounding)."""
    nside, lmax = 8, 16
    th, _ = healpix.pixel_angles(nside)
    c = synth.pol_small_case(th, lmax)
    c["cl4"][3] = 0.0
    d = polar.alm2map(c["signal_alm"], nside, lmax) + c["noise"]
    sched = synth.geometric_schedule(1e3, 4, 3)
    sp, ap = polar.solve(d, c["ninv6"], c["cl4"], sched, nside, lmax, mask=c["mask"])
    M = polar.ninv_matrices(c["ninv6"], c["mask"])
    # same tau for both: scale the T precision so its max equals the 3x3 maximum eigenvalue
    qt = M[:, 0, 0]
    s0, a0 = messenger.solve(d[0], qt, c["cl4"][0], sched, nside, lmax)
    tau_pol = polar.tau_of(M)
    if abs(tau_pol - messenger.tau_of(qt)) > 1e-15 * tau_pol:
        pytest.skip("tau set by the polarisation noise here")
    assert _rel(sp[0], s0) < 1e-13


def test_decoupled_temperature_with_shared_tau():
    """As above with a P noise that does not set tau: equal T results."""
    nside, lmax = 8, 16
    th, _ = healpix.pixel_angles(nside)
    c = synth.pol_small_case(th, lmax)
    c["cl4"][3] = 0.0
    n6 = c["ninv6"].copy()
    n6[1:] *= 0.2                      # P much noisier: tau comes from T
    d = polar.alm2map(c["signal_alm"], nside, lmax) + c["noise"]
    sched = synth.geometric_schedule(1e3, 4, 3)
    sp, ap = polar.solve(d, n6, c["cl4"], sched, nside, lmax, mask=c["mask"])
    qt = polar.ninv_matrices(n6, c["mask"])[:, 0, 0]
    s0, a0 = messenger.solve(d[0], qt, c["cl4"][0], sched, nside, lmax)
    assert _rel(sp[0], s0) < 1e-13
    assert _rel(ap[0], a0) < 1e-13


def test_uniform_fullsky_closed_form():
    """N^-1 = sigma^-2 1 on every pixel: W = 1, t = d at every sweep, so
    s_lm = F_l(lambda_last) map2alm(d)_lm with the 3x3 TE-coupled filter."""
    nside, lmax = 8, 16
    npx = 12 * nside * nside
    cl4 = synth.cl_pol(synth.cl_power_law(lmax))
    d = np.random.default_rng(9).standard_normal((3, npx)) * 30.0
    n6 = np.zeros((6, npx))
    n6[:3] = 1.0 / 900.0
    sched = [300.0, 20.0, 1.7]
    s_map, s_alm = polar.solve(d, n6, cl4, sched, nside, lmax)
    F = polar.harmonic_filter(cl4, 1.7, 900.0, healpix.pixel_area(nside))
    ref = polar.apply_filter(F, polar.map2alm(d, nside, lmax), lmax)
    assert _rel(s_alm, ref) < 1e-14
    assert _rel(s_map, polar.alm2map(ref, nside, lmax)) < 1e-14


def test_linearity_and_limits():
    nside, lmax = 4, 8
    th, _ = healpix.pixel_angles(nside)
    c = synth.pol_small_case(th, lmax)
    rs = np.random.default_rng(10)
    d1, d2 = rs.standard_normal((2, 3, 12 * nside * nside)) * 40
    sched = [100.0, 10.0, 1.0, 1.0]
    kw = dict(mask=c["mask"])
    a, _ = polar.solve(d1, c["ninv6"], c["cl4"], sched, nside, lmax, **kw)
    b, _ = polar.solve(d2, c["ninv6"], c["cl4"], sched, nside, lmax, **kw)
    ab, _ = polar.solve(2.0 * d1 - 0.5 * d2, c["ninv6"], c["cl4"], sched, nside, lmax, **kw)
    assert _rel(ab, 2.0 * a - 0.5 * b) < 1e-13
    big, _ = polar.solve(d1, c["ninv6"], c["cl4"], [1e30], nside, lmax, **kw)
    assert np.max(np.abs(big)) < 1e-20 * np.max(np.abs(d1))
    # no polarisation data and no TE: E = B = 0
    cl4 = c["cl4"].copy()
    cl4[3] = 0.0
    mask = (c["mask"] & 1).astype(np.uint8)
    _, al = polar.solve(d1, c["ninv6"], cl4, sched, nside, lmax, mask=mask)
    assert np.all(al[1:] == 0.0)


def _fp_case(nside=4, lmax=4):
    th, _ = healpix.pixel_angles(nside)
    c = synth.pol_small_case(th, lmax)
    d = polar.alm2map(c["signal_alm"], nside, lmax) + c["noise"]
    return c, d


@pytest.mark.parametrize("lam", [30.0, 3.0])
def test_dense_fixed_point_and_rate(lam):
    """At a fixed lambda the iteration converges geometrically to the dense fixed point
    at the rate of the iteration matrix's spectral radius (< 1)."""
    nside, lmax = 4, 4
    c, d = _fp_case(nside, lmax)
    fp_map, fp_alm = polar.messenger_fixed_point(d, c["ninv6"], c["cl4"], lam, nside, lmax, mask=c["mask"])
    G = polar.iteration_matrix(c["ninv6"], c["cl4"], lam, nside, lmax, mask=c["mask"])
    rho = float(np.max(np.abs(np.linalg.eigvals(G))))
    assert rho < 1.0
    errs = []
    M = polar.ninv_matrices(c["ninv6"], c["mask"])
    tau = polar.tau_of(M)
    s = np.zeros_like(d)
    for k in range(400):
        s, a = polar.sweep(s, d, M, c["cl4"], lam, tau, nside, lmax)
        errs.append(_rel(s, fp_map))
    assert errs[-1] < 1e-11 or errs[-1] < 2.0 * rho ** 400 * errs[0]
    k0, k1 = 40, 80
    if errs[k1] > 1e-12:
        rate = (errs[k1] / errs[k0]) ** (1.0 / (k1 - k0))
        assert rate <= rho * 1.05 + 1e-3


def test_fixed_point_at_lambda_one_near_wiener_filter():
    """At lambda = 1 the fixed point differs from Eq. (2) only by the quadrature defect
    of Omega Y^T Y (small at lmax = Nside)."""
    nside, lmax = 4, 4
    c, d = _fp_case(nside, lmax)
    fp, _ = polar.messenger_fixed_point(d, c["ninv6"], c["cl4"], 1.0, nside, lmax, mask=c["mask"])
    wf, _ = polar.wiener_dense(d, c["ninv6"], c["cl4"], nside, lmax, mask=c["mask"])
    assert _rel(fp, wf) < 0.05


def test_chi2_not_rising_at_fixed_lambda():
    """Coordinate descent on the joint objective: chi^2_lambda of the iterates does not
    rise by more than the quadrature defect allows."""
    nside, lmax = 8, 8
    th, _ = healpix.pixel_angles(nside)
    c = synth.pol_small_case(th, lmax)
    d = polar.alm2map(c["signal_alm"], nside, lmax) + c["noise"]
    M = polar.ninv_matrices(c["ninv6"], c["mask"])
    tau = polar.tau_of(M)
    lam = 5.0
    s = np.zeros_like(d)
    prev = None
    for k in range(30):
        s, a = polar.sweep(s, d, M, c["cl4"], lam, tau, nside, lmax)
        x = polar.chi2(s, a, d, M, c["cl4"], lmax, lam=lam, tau=tau)
        if prev is not None:
            assert x <= prev * (1.0 + 2e-3)
        prev = x
