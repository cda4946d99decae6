"""Adaptive cooling with band-limited transforms (oracle; test infrastructure only).

Elsner & Wandelt, Sect. 3. The messenger iteration of Sect. 2 is run with a
lambda that starts large and is lowered in steps:

  * lambda is tied to a multipole l_iter through the ratio of the messenger
    covariance to C_{l_iter}; it starts at l_iter = 20;
  * the chi^2 = s^dagger S^-1 s + (d - s)^dagger N^-1 (d - s) of the current
    iterate is the convergence monitor; once it has reached a plateau, l_iter is
    doubled and lambda set from the new l_iter;
  * the run ends at lambda = 1 once chi^2 improves by less than 1e-4 sigma_chi2
    from one iteration to the next;
  * while lambda smooths scales below l_iter away, the transforms of a sweep need
    only reach l_max^SHT, about l_iter + 100.

Readings adopted where the paper is silent (each listed in the design notes):
  * The ratio: lambda(l) = C_l / (tau Omega), the lambda at which the harmonic
    filter f_l(lambda) = C_l / (C_l + lambda tau Omega) is one half (the harmonic
    messenger covariance is tau Omega, see messenger.py). A level whose lambda
    would not exceed 1 (or whose l_iter exceeds lmax) is the last: lambda = 1.
  * l_max^SHT = min(lmax, l_iter + l_pad); the last level uses lmax itself, as
    the paper says the final iterations run at the full band limit.
  * sigma_chi2 = sqrt(2 n_obs), n_obs the observed pixels (chi^2 with n_obs
    degrees of freedom).
  * "Plateau": |chi2_{k-1} - chi2_k| < plateau_tol * sigma_chi2 for two iterates
    of the same level; a level also ends after max_level_sweeps sweeps (0: never).
  * Timing of the decisions: chi2 of iterate k is known once the map of iterate k
    has been synthesised, which happens at the start of sweep k + 1. A decision
    taken on chi2_k therefore applies from sweep k + 2 on; a stop leaves sweep
    k + 1 to finish and returns iterate k + 1.
  * A truncated sweep at band limit L is the sweep of messenger.py with the
    transform pair and the filter restricted to l <= L (the iterate has no modes
    above L; raising L adds modes that start at zero).
"""
import math

import numpy as np

from . import healpix
from .legendre import alm_index, n_alm
from .messenger import sweep, tau_of, chi2 as chi2_of


def levels(cl, lmax, tau, omega, l_iter0=20, l_pad=100, full_band=False):
    """[(lambda_j, L_j)] for l_iter = l_iter0 * 2^j; the last entry is (1, lmax)."""
    cl = np.asarray(cl, dtype=np.float64)
    out = []
    l_iter = l_iter0
    while True:
        ratio = cl[l_iter] / (tau * omega) if l_iter <= lmax else 0.0
        if ratio <= 1.0:
            out.append((1.0, lmax))
            return out
        band = lmax if full_band else min(lmax, l_iter + l_pad)
        out.append((float(ratio), band))
        l_iter *= 2


def pad_alm(alm, L, lmax):
    """Packed alm of band limit L in the packed layout of band limit lmax >= L."""
    out = np.zeros(n_alm(lmax), dtype=np.complex128)
    for m in range(L + 1):
        out[alm_index(lmax, m, m):alm_index(lmax, L, m) + 1] = alm[alm_index(L, m, m):alm_index(L, L, m) + 1]
    return out


def solve_banded(d, ninv, cl, lambdas, bands, nside, lmax, callback=None):
    """Sweep k at lambda lambdas[k] with the transforms cut at bands[k] (non-
    decreasing), from s = t = 0. Returns (s map, s alm in the lmax layout,
    [chi2 of every iterate at lambda = 1])."""
    ninv = np.asarray(ninv, dtype=np.float64)
    d = np.asarray(d, dtype=np.float64)
    cl = np.asarray(cl, dtype=np.float64)
    tau = tau_of(ninv)
    s_map = np.zeros(healpix.npix(nside))
    s_alm, band = np.zeros(1, dtype=np.complex128), 0
    chis = []
    for k, (lam, band) in enumerate(zip(lambdas, bands)):
        if k and band < bands[k - 1]:
            raise ValueError("band limits must not decrease")
        s_map, s_alm = sweep(s_map, d, ninv, cl[:band + 1], float(lam), tau, nside, band)
        chis.append(chi2_of(s_map, s_alm, d, ninv, cl[:band + 1], band, lam=1.0, tau=tau))
        if callback is not None:
            callback(k, s_map, s_alm)
    return s_map, pad_alm(s_alm, band, lmax), chis


def decide(k, lev, chis, cur, at_cur, nlevels, sigma, plateau_tol, stop_tol, max_level_sweeps):
    """The choice made once chi2 of iterate k is known (sweep k + 1 has started).

    lev[i] is the level of sweep i, chis[i] the chi2 of iterate i, cur the level of
    the latest sweep and at_cur the sweeps started at it. Returns (level of sweep
    k + 2, stop)."""
    final = cur == nlevels - 1
    nxt, stop = cur, False
    if k >= 1 and lev[k] == cur and lev[k - 1] == cur:
        gain = chis[k - 1] - chis[k]
        if final:
            stop = gain < stop_tol * sigma
        elif abs(gain) < plateau_tol * sigma:
            nxt = cur + 1
    if not final and max_level_sweeps > 0 and at_cur >= max_level_sweeps:
        nxt = cur + 1
    return nxt, stop


def solve_adaptive(d, ninv, cl, nside, lmax, max_sweeps, l_iter0=20, l_pad=100, full_band=False,
                   max_level_sweeps=50, plateau_tol=1.0, stop_tol=1e-4):
    """The adaptive schedule of Sect. 3 from s = t = 0.

    Returns (s map, s alm in the lmax layout, info) with info holding the lambda,
    band limit and chi2 of every sweep run and whether the stop rule ended it."""
    ninv = np.asarray(ninv, dtype=np.float64)
    d = np.asarray(d, dtype=np.float64)
    cl = np.asarray(cl, dtype=np.float64)
    tau = tau_of(ninv)
    lv = levels(cl, lmax, tau, healpix.pixel_area(nside), l_iter0, l_pad, full_band)
    sigma = math.sqrt(2.0 * np.count_nonzero(ninv > 0))
    lev = [0] * min(2, max_sweeps)          # levels of the sweeps started so far
    cur, at_cur, stopped = 0, len(lev), False
    chis = []
    s_map = np.zeros(healpix.npix(nside))
    s_alm, band = np.zeros(1, dtype=np.complex128), 0
    k = 0
    while k < len(lev):
        lam, band = lv[lev[k]]
        s_map, s_alm = sweep(s_map, d, ninv, cl[:band + 1], lam, tau, nside, band)
        chis.append(chi2_of(s_map, s_alm, d, ninv, cl[:band + 1], band, lam=1.0, tau=tau))
        if k + 1 < len(lev) and not stopped:
            nxt, stopped = decide(k, lev, chis, cur, at_cur, len(lv), sigma, plateau_tol, stop_tol,
                                  max_level_sweeps)
            if not stopped and len(lev) < max_sweeps:
                if nxt != cur:
                    cur, at_cur = nxt, 0
                lev.append(cur)
                at_cur += 1
        k += 1
    info = {"lambdas": np.array([lv[j][0] for j in lev]), "lmax_sht": np.array([lv[j][1] for j in lev]),
            "chi2": np.array(chis), "converged": stopped}
    return s_map, pad_alm(s_alm, band, lmax), info
