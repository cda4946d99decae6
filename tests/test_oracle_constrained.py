"""Pins of the oracle's constrained realisations (CPU only).

  * no fluctuation (xi = eta = 0) gives the Wiener filter itself;
  * s_CR(d) - s_CR(d') = WF(d) - WF(d') for the same draws (linearity);
  * with the exact Wiener filter of Eq. (2) (dense solve, Nside 4), over many draws
    for one data map the fluctuation s_CR - WF(d) has zero mean and, per l, the
    power of the posterior covariance (C^-1 + Y^T N^-1 Y)^-1 (Hoffman-Ribak);
  * with the data also drawn from the model, the realisations have the fiducial
    power (2l + 1) C_l per l: the unbiased spectrum of the paper's Sect. 3 figure.
"""
import numpy as np

from oracle import constrained, dense, healpix, messenger, sht
from oracle.legendre import alm_index
from paper_1211_0585_amd import synth
from tests.helpers import alm_rel_l2, rel_l2, small_band_inputs


def test_zero_draws_give_the_wiener_filter():
    nside, lmax = 8, 16
    c = small_band_inputs(nside, lmax, seed=2)
    lams = np.geomspace(100.0, 1.0, 12)
    xi = np.zeros((lmax + 1) * (lmax + 2) // 2, dtype=np.complex128)
    eta = np.zeros(healpix.npix(nside))
    m, a = constrained.constrained_messenger(c["d"], c["ninv"], c["cl"], xi, eta, lams, nside, lmax)
    m0, a0 = messenger.solve(c["d"], c["ninv"], c["cl"], lams, nside, lmax)
    assert np.array_equal(m, m0) and np.array_equal(a, a0)


def test_linear_in_the_data():
    nside, lmax = 8, 16
    c = small_band_inputs(nside, lmax, seed=3)
    c2 = small_band_inputs(nside, lmax, seed=4)
    lams = np.geomspace(100.0, 1.0, 12)
    xi, eta = synth.fluctuation_draws(healpix.npix(nside), lmax, 5)
    m1, a1 = constrained.constrained_messenger(c["d"], c["ninv"], c["cl"], xi[0], eta[0], lams, nside, lmax)
    m2, a2 = constrained.constrained_messenger(c2["d"], c["ninv"], c["cl"], xi[0], eta[0], lams, nside, lmax)
    w1, b1 = messenger.solve(c["d"], c["ninv"], c["cl"], lams, nside, lmax)
    w2, b2 = messenger.solve(c2["d"], c["ninv"], c["cl"], lams, nside, lmax)
    assert rel_l2(m1 - m2, w1 - w2) < 1e-12
    assert alm_rel_l2(a1 - a2, b1 - b2, lmax) < 1e-12


def test_signal_draw_has_unit_scaled_power():
    lmax = 6
    cl = np.arange(lmax + 1, dtype=float) ** 2
    xi = np.arange(1, (lmax + 1) * (lmax + 2) // 2 + 1) * (1.0 + 2.0j)
    a = constrained.signal_draw_alm(cl, xi, lmax)
    for m in range(lmax + 1):
        for l in range(m, lmax + 1):
            i = alm_index(lmax, l, m)
            want = np.sqrt(cl[l]) * (xi[i].real if m == 0 else xi[i])
            assert a[i] == want
    eta = np.array([1.0, -2.0, 3.0])
    assert np.array_equal(constrained.noise_draw(np.array([4.0, 0.0, 0.25]), eta), np.array([0.5, 0.0, 6.0]))


def _dense_setup(nside, lmax, c):
    modes = dense.real_modes(lmax, c["cl"])
    Y = dense.synthesis_matrix(nside, lmax, modes)
    Cd = np.array([c["cl"][l] for (l, _, _) in modes])
    A = np.diag(1.0 / Cd) + Y.T @ (c["ninv"][:, None] * Y)
    K = np.linalg.solve(A, Y.T * c["ninv"])              # x = K d: Eq. (2) in the real basis
    post = np.linalg.inv(A)                               # posterior covariance

    def wf(dd):
        x = K @ dd
        return Y @ x, dense.x_to_alm(x, modes, lmax)
    return modes, post, wf


def _power_per_l(a, lmax):
    w = sht.alm_weights(lmax)
    ell = sht.alm_ell(lmax)
    return np.array([np.sum(w[ell == l] * np.abs(a[ell == l]) ** 2) for l in range(lmax + 1)])


def test_fluctuations_have_posterior_covariance():
    nside, lmax = 4, 4
    c = small_band_inputs(nside, lmax, seed=6)
    modes, post, wf = _dense_setup(nside, lmax, c)
    _, a_wf = wf(c["d"])
    ndraw = 3000
    xi, eta = synth.fluctuation_draws(healpix.npix(nside), lmax, 11, nmaps=ndraw)
    P = np.empty((ndraw, lmax + 1))
    mean = np.zeros_like(a_wf)
    for i in range(ndraw):
        _, a = constrained.constrained(c["d"], c["ninv"], c["cl"], xi[i], eta[i], nside, lmax, wf)
        P[i] = _power_per_l(a - a_wf, lmax)
        mean += (a - a_wf) / ndraw
    tr = np.zeros(lmax + 1)
    for k, (l, _, _) in enumerate(modes):
        tr[l] += post[k, k]
    for l in range(2, lmax + 1):
        err = P[:, l].std() / np.sqrt(ndraw)
        assert abs(P[:, l].mean() - tr[l]) < 4 * err, (l, P[:, l].mean(), tr[l], err)
    # zero mean: each entry within 4 sigma of its posterior spread
    ell = sht.alm_ell(lmax)
    for l in range(2, lmax + 1):
        spread = np.sqrt(tr[l] / (2 * l + 1))
        assert np.all(np.abs(mean[ell == l]) < 4 * spread / np.sqrt(ndraw) * 1.5)


def test_realisations_have_the_fiducial_spectrum():
    nside, lmax = 4, 4
    c = small_band_inputs(nside, lmax, seed=7)
    _, _, wf = _dense_setup(nside, lmax, c)
    ndraw = 3000
    npix = healpix.npix(nside)
    xi, eta = synth.fluctuation_draws(npix, lmax, 12, nmaps=ndraw)
    xs, es = synth.fluctuation_draws(npix, lmax, 13, nmaps=ndraw)   # the data's own signal and noise
    P = np.empty((ndraw, lmax + 1))
    for i in range(ndraw):
        d = sht.alm2map(constrained.signal_draw_alm(c["cl"], xs[i], lmax), nside, lmax) \
            + constrained.noise_draw(c["ninv"], es[i])
        _, a = constrained.constrained(d, c["ninv"], c["cl"], xi[i], eta[i], nside, lmax, wf)
        P[i] = _power_per_l(a, lmax)
    for l in range(2, lmax + 1):
        want = (2 * l + 1) * c["cl"][l]
        err = P[:, l].std() / np.sqrt(ndraw)
        assert abs(P[:, l].mean() - want) < 4 * err, (l, P[:, l].mean(), want, err)
