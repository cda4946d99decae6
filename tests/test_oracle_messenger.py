"""Pins of the oracle's messenger iteration and dense solves (CPU only).

  * the per-pixel and per-mode solutions of Eqs. (3) and (4) against the
    equations themselves written with Nbar = N - T and T = tau;
  * the full-sky uniform-noise special case, where w = 1 and the result after
    any number of sweeps is f_l(lambda_last) * map2alm(d) exactly;
  * linearity in d and the lambda -> infinity limit;
  * the dense fixed point at fixed lambda (geometric convergence at the rate of
    the iteration matrix's spectral radius, which is < 1: Sect. 2);
  * the textbook Wiener filter (Eq. 2) against its Woodbury form;
  * chi^2_lambda non-increasing per sweep (within the quadrature defect) and
    chi^2_min / n_obs ~ 1 (Sect. 3, Fig. 2).
"""
import numpy as np
import pytest

from oracle import dense, healpix, messenger, sht
from oracle.legendre import n_alm
from paper_1211_0585_amd import synth


def _small_case(nside, lmax, seed=0):
    theta, phi = healpix.pixel_angles(nside)
    c = synth.small_band_case(theta, lmax, seed=seed)
    s = sht.alm2map(c["signal_alm"], nside, lmax)
    c["d"] = s + c["noise"]
    return c


def test_pixel_step_solves_eq3():
    """t = s + w (d - s) solves (Nbar^-1 + (lambda T)^-1) t = Nbar^-1 d + (lambda T)^-1 s."""
    rs = np.random.default_rng(0)
    ninv = rs.uniform(0.2, 5.0, 1000)
    tau = messenger.tau_of(ninv)
    d, s = rs.standard_normal(1000), rs.standard_normal(1000)
    for lam in (1.0, 3.7, 1e4):
        w = messenger.pixel_weight(ninv, lam, tau)
        t = s + w * (d - s)
        nbar = 1.0 / ninv - tau
        ok = nbar > 1e-12 * tau                    # the min-noise pixel has Nbar = 0
        lhs = (1.0 / nbar[ok] + 1.0 / (lam * tau)) * t[ok]
        rhs = d[ok] / nbar[ok] + s[ok] / (lam * tau)
        assert np.allclose(lhs, rhs, rtol=1e-12, atol=0)
        assert np.all((w >= 0) & (w <= 1))
        assert abs(w[np.argmax(ninv)] - 1.0) < 1e-15   # Nbar = 0 -> t = d
    # masked pixel: ninv = 0 -> Nbar infinite -> t = s
    assert messenger.pixel_weight(np.array([0.0]), 7.0, 0.3)[0] == 0.0


def test_harmonic_step_solves_eq4():
    """s = f t solves (S^-1 + (lambda T_h)^-1) s = (lambda T_h)^-1 t with T_h = tau Omega."""
    cl = synth.cl_power_law(64)
    tau, omega = 0.37, healpix.pixel_area(16)
    for lam in (1.0, 20.0, 1e4):
        f = messenger.harmonic_filter(cl, lam, tau, omega)
        t = np.random.default_rng(1).standard_normal(65)
        s = f * t
        th = lam * tau * omega
        assert np.allclose((1.0 / cl[2:] + 1.0 / th) * s[2:], t[2:] / th, rtol=1e-13, atol=0)
        assert np.all(f[:2] == 0.0)


@pytest.mark.parametrize("nside,lmax,nsweeps", [(8, 16, 1), (16, 32, 3)])
def test_fullsky_uniform_noise_closed_form(nside, lmax, nsweeps):
    """I8: uniform full-sky noise => w = 1 => s_lm = C_l/(C_l + lambda sigma^2 Omega) d_lm."""
    c = synth.uniform_fullsky_case(healpix.npix(nside), lmax, sigma_muk=30.0, n_sweeps=nsweeps)
    d = sht.alm2map(c["signal_alm"], nside, lmax) + c["noise"]
    lams = c["schedule"]
    s_map, s_alm = messenger.solve(d, c["ninv"], c["cl"], lams, nside, lmax)
    sig2, omega = 30.0 ** 2, healpix.pixel_area(nside)
    cl = c["cl"]
    f = np.where(cl > 0, cl / (cl + lams[-1] * sig2 * omega), 0.0)
    want = messenger.expand_l(f, lmax) * sht.map2alm(d, nside, lmax)
    assert np.allclose(s_alm, want, rtol=0, atol=1e-14 * np.abs(want).max())
    assert np.allclose(s_map, sht.alm2map(want, nside, lmax), rtol=0, atol=1e-13 * np.abs(s_map).max())


def test_linearity_and_limits():
    """I12: solve(a d1 + b d2) = a solve(d1) + b solve(d2); lambda -> inf gives s -> 0."""
    nside, lmax = 8, 16
    c1 = _small_case(nside, lmax, seed=1)
    c2 = _small_case(nside, lmax, seed=2)
    lams = synth.geometric_schedule(1e3, 5, 5)
    s1, a1 = messenger.solve(c1["d"], c1["ninv"], c1["cl"], lams, nside, lmax)
    s2, a2 = messenger.solve(c2["d"], c1["ninv"], c1["cl"], lams, nside, lmax)
    s12, a12 = messenger.solve(2.0 * c1["d"] - 0.5 * c2["d"], c1["ninv"], c1["cl"], lams, nside, lmax)
    ref = 2.0 * s1 - 0.5 * s2
    assert np.linalg.norm(s12 - ref) <= 1e-13 * np.linalg.norm(ref)
    sbig, _ = messenger.solve(c1["d"], c1["ninv"], c1["cl"], [1e30], nside, lmax)
    assert np.abs(sbig).max() < 1e-20 * np.abs(c1["d"]).max()


def test_first_sweep_is_filtered_weighted_data():
    """From s = t = 0 (Sect. 2), the first sweep gives t = w d."""
    nside, lmax = 8, 16
    c = _small_case(nside, lmax)
    lam = 50.0
    tau = messenger.tau_of(c["ninv"])
    _, a = messenger.solve(c["d"], c["ninv"], c["cl"], [lam], nside, lmax)
    t = messenger.pixel_weight(c["ninv"], lam, tau) * c["d"]
    f = messenger.harmonic_filter(c["cl"], lam, tau, healpix.pixel_area(nside))
    want = messenger.expand_l(f, lmax) * sht.map2alm(t, nside, lmax)
    assert np.allclose(a, want, rtol=0, atol=1e-15 * np.abs(want).max())


def _iterate_fixed(c, lam, nside, lmax, n):
    tau = messenger.tau_of(c["ninv"])
    s = np.zeros(healpix.npix(nside))
    hist = []
    for _ in range(n):
        s, a = messenger.sweep(s, c["d"], c["ninv"], c["cl"], lam, tau, nside, lmax)
        hist.append(a)
    return s, hist


@pytest.mark.parametrize("nside,lmax", [(4, 4), (8, 8)])
def test_dense_fixed_point_and_convergence_rate(nside, lmax):
    """I9: iterating at fixed lambda converges to the dense fixed point, with
    error decaying geometrically at the spectral radius of the iteration matrix."""
    c = _small_case(nside, lmax, seed=5)
    for lam in (100.0, 10.0, 1.0):
        M = dense.iteration_matrix(c["ninv"], c["cl"], lam, nside, lmax)
        rho = float(np.max(np.abs(np.linalg.eigvals(M))))
        assert rho < 1.0
        s_star, a_star = dense.messenger_fixed_point(c["d"], c["ninv"], c["cl"], lam, nside, lmax)
        n = int(min(4000, max(60, np.ceil(np.log(1e-14) / np.log(rho)) + 20)))
        s, hist = _iterate_fixed(c, lam, nside, lmax, n)
        w = sht.alm_weights(lmax)
        err = [np.sqrt(np.sum(w * np.abs(h - a_star) ** 2)) for h in hist]
        ref = np.sqrt(np.sum(w * np.abs(a_star) ** 2))
        assert err[-1] <= 1e-11 * ref, (lam, rho, err[-1] / ref)
        assert np.linalg.norm(s - s_star) <= 1e-11 * np.linalg.norm(s_star)
        # observed asymptotic rate matches rho
        k0 = len(err) // 3
        k1 = next((k for k in range(k0, len(err)) if err[k] < 1e-9 * ref), len(err) - 1)
        if k1 - k0 > 10 and err[k0] > 0:
            rate = (err[k1] / err[k0]) ** (1.0 / (k1 - k0))
            assert abs(rate - rho) < 0.05 + 0.1 * (1 - rho), (lam, rate, rho)


def test_wiener_dense_woodbury():
    """Eq. (2) solved in harmonic space equals the data-space (Woodbury) form
    x = C Y_o^T (Y_o C Y_o^T + N_o)^-1 d_o over the observed pixels."""
    nside, lmax = 4, 6
    c = _small_case(nside, lmax, seed=9)
    s_map, a = dense.wiener_dense(c["d"], c["ninv"], c["cl"], nside, lmax)
    modes = dense.real_modes(lmax, c["cl"])
    Y = dense.synthesis_matrix(nside, lmax, modes)
    obs = c["ninv"] > 0
    Cd = np.array([c["cl"][l] for (l, _, _) in modes])
    Yo = Y[obs]
    K = (Yo * Cd) @ Yo.T + np.diag(1.0 / c["ninv"][obs])
    x = Cd * (Yo.T @ np.linalg.solve(K, c["d"][obs]))
    assert np.allclose(Y @ x, s_map, rtol=0, atol=1e-11 * np.abs(s_map).max())
    assert np.allclose(dense.x_to_alm(x, modes, lmax), a, rtol=0, atol=1e-11 * np.abs(a).max())


def test_quadrature_gap_shrinks_with_nside():
    """At lambda = 1 the messenger fixed point differs from Eq. (2) only through
    Omega Y^T Y != I; that gap shrinks as Nside grows at fixed lmax."""
    lmax = 4
    gaps = []
    for nside in (4, 8, 16):
        c = _small_case(nside, lmax, seed=3)
        s1, _ = dense.wiener_dense(c["d"], c["ninv"], c["cl"], nside, lmax)
        s2, _ = dense.messenger_fixed_point(c["d"], c["ninv"], c["cl"], 1.0, nside, lmax)
        gaps.append(np.linalg.norm(s2 - s1) / np.linalg.norm(s1))
    assert gaps[0] > gaps[1] > gaps[2]
    assert gaps[2] < 1e-2


def test_gram_defect_nside1_by_hand():
    """Nside 1 (rings z = 2/3, 0, -2/3, four pixels each, Omega = pi/3), worked by hand:
    at lmax 0 the monopole is exact (Omega * 12 / (4 pi) = 1); at lmax 1 the Gram matrix
    of (Y_00, Y_10, Y_11^c, Y_11^s) is diag(1, 8/9, 19/18, 19/18): sum z^2 = 32/9 times
    3/(4 pi) Omega gives 8/9; sum sin^2(theta) cos^2(phi) = 2 (5/9) 2 + 2 = 38/9 gives 19/18;
    every cross term sums to zero over a ring. So ||I - G||_2 = 1/9."""
    assert dense.gram_defect(1, 0) < 1e-15
    G, modes = dense.gram_matrix(1, 1)
    assert modes == [(0, 0, 0), (1, 0, 0), (1, 1, 1), (1, 1, 2)]
    assert np.allclose(G, np.diag([1.0, 8.0 / 9.0, 19.0 / 18.0, 19.0 / 18.0]), rtol=0, atol=1e-15)
    assert abs(dense.gram_defect(1, 1) - 1.0 / 9.0) < 1e-15


@pytest.mark.parametrize("nside,lmax", [(1, 3), (2, 6), (4, 8), (8, 12)])
def test_gram_trace_is_addition_theorem(nside, lmax):
    """trace of the l-block of Omega Y^T Y = Omega npix (2l+1)/(4 pi) = 2l + 1 exactly
    (addition theorem at every pixel), so I - G has eigenvalues of both signs."""
    G, modes = dense.gram_matrix(nside, lmax)
    ell = np.array([l for (l, _, _) in modes])
    for l in range(lmax + 1):
        assert abs(np.trace(G[np.ix_(ell == l, ell == l)]) - (2 * l + 1)) < 1e-12 * (2 * l + 1)
    ev = np.linalg.eigvalsh(np.eye(len(modes)) - G)
    assert abs(max(abs(ev.min()), abs(ev.max())) - dense.gram_defect(nside, lmax)) < 1e-14
    if nside * 2 <= lmax:
        assert ev.min() < 0 < ev.max()


def test_chi2_monotone_at_fixed_lambda():
    """I10: chi^2_lambda(s) is non-increasing per sweep at fixed lambda up to the
    quadrature defect || I - Omega Y^T Y ||."""
    nside, lmax = 16, 8
    defect = dense.gram_defect(nside, lmax)
    assert defect < 1e-2
    c = _small_case(nside, lmax, seed=4)
    tau = messenger.tau_of(c["ninv"])
    for lam in (30.0, 1.0):
        s = np.zeros(healpix.npix(nside))
        prev = None
        for _ in range(40):
            s, a = messenger.sweep(s, c["d"], c["ninv"], c["cl"], lam, tau, nside, lmax)
            x2 = messenger.chi2(s, a, c["d"], c["ninv"], c["cl"], lmax, lam=lam, tau=tau)
            if prev is not None:
                assert x2 <= prev * (1.0 + defect), (lam, x2, prev)
            prev = x2


def test_chi2_min_matches_dof():
    """I11: for data drawn from the model, chi^2 at the Wiener solution is
    chi^2-distributed with n_obs degrees of freedom (Sect. 3: chi^2/n_dof ~ 1)."""
    nside, lmax = 8, 12
    vals = []
    for seed in range(4):
        c = _small_case(nside, lmax, seed=seed)
        s_map, a = dense.wiener_dense(c["d"], c["ninv"], c["cl"], nside, lmax)
        x2 = messenger.chi2(s_map, a, c["d"], c["ninv"], c["cl"], lmax)
        vals.append(x2 / np.count_nonzero(c["ninv"]))
    nobs = np.count_nonzero(_small_case(nside, lmax)["ninv"])
    sig = np.sqrt(2.0 / nobs) / np.sqrt(len(vals))
    assert abs(np.mean(vals) - 1.0) < 4 * sig, (vals, sig)


def test_alm_packing_size():
    assert n_alm(32) == 561 and n_alm(1024) == 525825
