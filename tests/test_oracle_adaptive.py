"""Pins of the oracle's adaptive schedule and band-limited sweeps (CPU only), and
the library's host-side level table against it.

  * the level table: lambda_j makes f_{l_j}(lambda_j) = 1/2 (the ratio reading of
    Sect. 3), l_iter doubles, the band limit is l_iter + margin, and the last
    level has lambda 1 at the full band limit; the C ABI's table is identical;
  * a sweep with the transforms cut at L equals the full-band sweep with C_l set
    to zero above L (the iterate then has no modes above L), for single sweeps
    and for whole schedules with rising band limits;
  * the decision rules (plateau, stop, level cap, one-sweep lag) on scripted
    chi^2 sequences;
  * the adaptive run converges to the dense fixed point at lambda = 1 (Sect. 2),
    chi^2 does not rise at the last level (up to the quadrature defect), and its
    final chi^2 / n_obs is about 1 (Sect. 3).
"""
import math

import numpy as np
import pytest

from oracle import adaptive, dense, healpix, messenger
from tests.helpers import alm_rel_l2, rel_l2, small_band_inputs


def _case(nside, lmax, seed=0):
    return small_band_inputs(nside, lmax, seed=seed)


def test_levels_closed_form():
    nside, lmax = 16, 32
    c = _case(nside, lmax)
    tau, om = messenger.tau_of(c["ninv"]), healpix.pixel_area(nside)
    lv = adaptive.levels(c["cl"], lmax, tau, om, l_iter0=2, l_pad=4)
    assert lv[-1] == (1.0, lmax)
    for j, (lam, band) in enumerate(lv[:-1]):
        l_iter = 2 << j
        f = messenger.harmonic_filter(c["cl"], lam, tau, om)[l_iter]
        assert abs(f - 0.5) < 1e-15 and lam > 1.0
        assert band == min(lmax, l_iter + 4)
    # the level after the last non-final one has ratio <= 1 (or lies above lmax)
    l_next = 2 << (len(lv) - 1)
    assert l_next > lmax or c["cl"][l_next] / (tau * om) <= 1.0
    assert all(a[0] >= b[0] for a, b in zip(lv, lv[1:]))
    full = adaptive.levels(c["cl"], lmax, tau, om, l_iter0=2, l_pad=4, full_band=True)
    assert [b for _, b in full] == [lmax] * len(full)
    assert [x for x, _ in full] == [x for x, _ in lv]


@pytest.mark.parametrize("l0,pad,full", [(2, 4, 0), (20, 100, 0), (3, 0, 0), (2, 4, 1), (64, 10, 0)])
def test_host_level_table_matches_oracle(l0, pad, full):
    """wf_adaptive_levels (host-only C ABI) against the oracle's table."""
    from paper_1211_0585_amd import mwf
    lmax = 40
    c = _case(16, lmax, seed=2)
    tau, om = messenger.tau_of(c["ninv"]), healpix.pixel_area(16)
    ref = adaptive.levels(c["cl"], lmax, tau, om, l_iter0=l0, l_pad=pad, full_band=bool(full))
    got = mwf.adaptive_levels(lmax, c["cl"], tau, om, l_iter0=l0, l_pad=pad, full_band=full)
    assert got == ref


def test_host_level_table_rejects_bad_options():
    from paper_1211_0585_amd import mwf
    cl = np.ones(9)
    for kw in ({"l_iter0": 0}, {"l_pad": -1}, {"full_band": 2}, {"plateau_tol": -1.0},
               {"stop_tol": float("nan")}, {"max_level_sweeps": -3}):
        with pytest.raises(mwf.WFError) as e:
            mwf.adaptive_levels(8, cl, 1.0, 0.1, **kw)
        assert e.value.code == mwf.WF_EINVAL
    with pytest.raises(mwf.WFError):
        mwf.adaptive_levels(8, cl, 0.0, 0.1)


@pytest.mark.parametrize("band", [0, 3, 9])
def test_truncated_sweep_is_sweep_with_zeroed_cl(band):
    nside, lmax = 8, 16
    c = _case(nside, lmax, seed=1)
    tau = messenger.tau_of(c["ninv"])
    s0 = np.random.default_rng(3).standard_normal(healpix.npix(nside))   # any iterate, any modes
    cz = c["cl"].copy()
    cz[band + 1:] = 0.0
    for lam in (40.0, 1.0):
        m_t, a_t = messenger.sweep(s0, c["d"], c["ninv"], c["cl"][:band + 1], lam, tau, nside, band)
        m_f, a_f = messenger.sweep(s0, c["d"], c["ninv"], cz, lam, tau, nside, lmax)
        if np.linalg.norm(m_f) == 0:
            assert np.linalg.norm(m_t) == 0
            continue
        assert rel_l2(m_t, m_f) < 1e-13
        assert alm_rel_l2(adaptive.pad_alm(a_t, band, lmax), a_f, lmax) < 1e-13


def test_banded_schedule_is_schedule_with_zeroed_cl():
    nside, lmax = 16, 24
    c = _case(nside, lmax, seed=4)
    tau = messenger.tau_of(c["ninv"])
    lams = [300.0, 120.0, 120.0, 30.0, 30.0, 8.0, 1.0, 1.0]
    bands = [4, 6, 6, 10, 10, 16, 24, 24]
    m_b, a_b, chis = adaptive.solve_banded(c["d"], c["ninv"], c["cl"], lams, bands, nside, lmax)
    s = np.zeros(healpix.npix(nside))
    for k, (lam, band) in enumerate(zip(lams, bands)):
        cz = c["cl"].copy()
        cz[band + 1:] = 0.0
        s, a = messenger.sweep(s, c["d"], c["ninv"], cz, lam, tau, nside, lmax)
        assert abs(chis[k] - messenger.chi2(s, a, c["d"], c["ninv"], cz, lmax, tau=tau)) < 1e-11 * chis[k]
    assert rel_l2(m_b, s) < 1e-12
    assert alm_rel_l2(a_b, a, lmax) < 1e-12
    # full band everywhere: the plain solve
    m_p, a_p = messenger.solve(c["d"], c["ninv"], c["cl"], lams, nside, lmax)
    m_q, a_q, _ = adaptive.solve_banded(c["d"], c["ninv"], c["cl"], lams, [lmax] * len(lams), nside, lmax)
    assert rel_l2(m_q, m_p) < 1e-15 and alm_rel_l2(a_q, a_p, lmax) < 1e-15
    with pytest.raises(ValueError):
        adaptive.solve_banded(c["d"], c["ninv"], c["cl"], [1.0, 1.0], [8, 4], nside, lmax)


def test_decide_rules():
    d = adaptive.decide
    kw = dict(nlevels=3, sigma=10.0, plateau_tol=1.0, stop_tol=0.01, max_level_sweeps=0)
    # plateau needs two iterates of the current level
    assert d(0, [0, 0], [500.0], 0, 2, **kw) == (0, False)
    assert d(1, [0, 0, 0], [500.0, 420.0], 0, 3, **kw) == (0, False)
    assert d(1, [0, 0, 0], [500.0, 491.0], 0, 3, **kw) == (1, False)      # |D| = 9 < 10
    assert d(1, [0, 0, 0], [500.0, 509.5], 0, 3, **kw) == (1, False)      # rising also plateaus
    # iterate k - 1 belongs to the previous level: no test
    assert d(3, [0, 0, 0, 1, 1], [9.0, 8.0, 7.0, 6.99], 1, 2, **kw) == (1, False)
    assert d(4, [0, 0, 0, 1, 1, 1], [9.0, 8.0, 7.0, 6.99, 6.98], 1, 3, **kw) == (2, False)
    # last level: stop on a gain below stop_tol * sigma (0.1), not on a plateau
    assert d(6, [2] * 8, [0] * 5 + [50.0, 49.95], 2, 8, **kw) == (2, True)
    assert d(6, [2] * 8, [0] * 5 + [50.0, 49.5], 2, 8, **kw) == (2, False)
    assert d(6, [2] * 8, [0] * 5 + [50.0, 50.2], 2, 8, **kw) == (2, True)  # no gain at all
    # level cap, but never past the last level
    cap = dict(kw, max_level_sweeps=4)
    assert d(2, [0] * 4, [900.0, 700.0, 500.0], 0, 4, **cap) == (1, False)
    assert d(2, [0] * 4, [900.0, 700.0, 500.0], 0, 3, **cap) == (0, False)
    assert d(9, [2] * 11, [0] * 8 + [60.0, 40.0], 2, 40, **cap) == (2, False)


def test_schedule_on_scripted_chi2(monkeypatch):
    """The control flow of solve_adaptive with the sweep stubbed out and a scripted
    chi^2 per iterate: decisions taken on iterate k steer sweep k + 2."""
    script = iter([100.0, 99.5,            # iterates 0, 1 (level 0): plateau seen at k = 1
                   98.0,                   # iterate 2 still level 0 (sweep 2 was already running)
                   60.0, 40.0, 39.8,       # level 1 from sweep 3; plateau at k = 5
                   39.0,                   # iterate 6: level 1
                   30.0, 29.99995,         # level 2 (last) from sweep 7; stop at k = 8
                   29.9999, 0.0])          # iterate 9 is the result
    monkeypatch.setattr(adaptive, "sweep", lambda s, d, ninv, cl, lam, tau, nside, band: (s, np.zeros(1)))
    monkeypatch.setattr(adaptive, "chi2_of", lambda *a, **k: next(script))
    monkeypatch.setattr(adaptive, "pad_alm", lambda a, L, lmax: a)
    cl = np.zeros(41)
    cl[2:] = 8.0 / np.arange(2, 41) ** 2     # ratio C_l / Omega: 7.6 at l = 2, 1.9 at 4, 0.48 at 8
    ninv = np.ones(healpix.npix(2))
    omega = healpix.pixel_area(2)
    # tau = 1; levels at l = 2, 4 (ratio > 1) and the last one
    lv = adaptive.levels(cl, 40, 1.0, omega, l_iter0=2, l_pad=1)
    assert len(lv) == 3 and lv[1][0] > 1.0
    sigma = math.sqrt(2.0 * 48)
    _, _, info = adaptive.solve_adaptive(np.zeros(48), ninv, cl, 2, 40, 50, l_iter0=2, l_pad=1,
                                         plateau_tol=1.0 / sigma, stop_tol=1e-3 / sigma, max_level_sweeps=0)
    assert info["converged"]
    assert [b for b in info["lmax_sht"]] == [3, 3, 3, 5, 5, 5, 5, 40, 40, 40]
    assert len(info["chi2"]) == 10
    # the sweep cap ends a run early, without convergence
    script = iter([100.0, 99.5, 98.0, 60.0, 40.0, 39.8, 39.0])
    monkeypatch.setattr(adaptive, "chi2_of", lambda *a, **k: next(script))
    _, _, info = adaptive.solve_adaptive(np.zeros(48), ninv, cl, 2, 40, 5, l_iter0=2, l_pad=1,
                                         plateau_tol=1.0 / sigma, stop_tol=1e-3 / sigma, max_level_sweeps=0)
    assert not info["converged"] and list(info["lmax_sht"]) == [3, 3, 3, 5, 5]


def test_adaptive_reaches_dense_fixed_point():
    """With a tight stop rule the adaptive run ends at the lambda = 1 fixed point of
    the sweep (dense solve, Sect. 2). The stop rule ends a run at the first
    iteration whose chi^2 gain falls below the tolerance; where the quadrature
    defect lets chi^2 rise near the end (lmax > nside here) that happens early, so
    the case keeps lmax = nside."""
    nside, lmax = 8, 8
    c = _case(nside, lmax, seed=5)
    s_star, a_star = dense.messenger_fixed_point(c["d"], c["ninv"], c["cl"], 1.0, nside, lmax)
    s, a, info = adaptive.solve_adaptive(c["d"], c["ninv"], c["cl"], nside, lmax, 3000, l_iter0=2, l_pad=2,
                                         plateau_tol=0.01, stop_tol=1e-12, max_level_sweeps=0)
    assert info["converged"]
    assert list(info["lmax_sht"])[-1] == lmax and info["lambdas"][-1] == 1.0
    assert min(info["lmax_sht"]) < lmax
    assert rel_l2(s, s_star) < 1e-6
    assert alm_rel_l2(a, a_star, lmax) < 1e-6


def test_adaptive_chi2_at_last_level():
    """chi^2 does not rise at the last level beyond the quadrature defect (I10),
    and the final chi^2 / n_obs lies within 4 sigma of 1 (Sect. 3, Fig. 2)."""
    nside, lmax = 16, 32
    c = _case(nside, lmax, seed=0)
    defect = dense.gram_defect(nside, 8)
    s, a, info = adaptive.solve_adaptive(c["d"], c["ninv"], c["cl"], nside, lmax, 300, l_iter0=2, l_pad=4)
    assert info["converged"]
    lv = info["lambdas"]
    chi = info["chi2"]
    last = [k for k in range(len(lv)) if lv[k] == 1.0]
    assert len(set(info["lmax_sht"][:last[0]])) > 2          # several truncated levels before
    for k0, k1 in zip(last, last[1:]):
        assert chi[k1] <= chi[k0] * (1.0 + defect)
    nobs = np.count_nonzero(c["ninv"])
    assert abs(chi[-1] / nobs - 1.0) < 4 * math.sqrt(2.0 / nobs)
    # the reported chi^2 is that of the returned iterate
    assert abs(messenger.chi2(s, a, c["d"], c["ninv"], c["cl"], lmax) - chi[-1]) < 1e-10 * chi[-1]
