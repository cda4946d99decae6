"""Messenger-field iteration (oracle; test infrastructure only).

Elsner & Wandelt, Sect. 2. With data d = s + n (Eq. 1) the Wiener filter solves
(S^-1 + N^-1) s = N^-1 d (Eq. 2). A messenger field t with covariance T = tau*1,
tau = min(diag N) (Sect. 2, below Eq. 4), and Nbar = N - T give the pair

  Eq. (3)  (Nbar^-1 + (lambda T)^-1) t = Nbar^-1 d + (lambda T)^-1 s   (pixel basis)
  Eq. (4)  (S^-1 + (lambda T)^-1) s = (lambda T)^-1 t                  (harmonic basis)

iterated from s = t = 0: solve (3) for t in the noise basis, change basis,
solve (4) for s, change back (Sect. 2, outline of the algorithm). At lambda = 1
the pair reduces to Eq. (2).

Readings adopted where the paper is silent (each listed in the design notes):
  * N is diagonal in pixels with N^-1_p = ninv[p] >= 0; ninv = 0 marks a masked
    (unobserved) pixel, i.e. infinite noise; tau = 1 / max_p ninv[p].
  * Eq. (3) per pixel, with Nbar_p = 1/ninv_p - tau, is rewritten without any
    division by zero as t_p = s_p + w_p (d_p - s_p),
        w_p = lambda tau ninv_p / (1 + (lambda - 1) tau ninv_p)  (w = 0 if masked).
  * In harmonic space the messenger covariance is tau * Omega (white pixel
    noise of variance tau has alm variance tau * Omega under the analysis
    Omega Y^dagger), so Eq. (4) per mode is s_lm = f_l a_lm,
        f_l = C_l / (C_l + lambda tau Omega),  f_l = 0 where C_l = 0.
  * One sweep = t-step, analysis, s-step, synthesis; the output is the final
    synthesised map s and its alm.
"""
import numpy as np

from . import healpix, sht
from .legendre import alm_index, n_alm


def tau_of(ninv):
    """tau = min over observed pixels of diag N = 1 / max ninv (Sect. 2)."""
    ninv = np.asarray(ninv, dtype=np.float64)
    mx = ninv.max()
    if not mx > 0:
        raise ValueError("no observed pixel (all ninv == 0)")
    return 1.0 / mx


def pixel_weight(ninv, lam, tau):
    """w_p(lambda): the pixel-space solution of Eq. (3) is t = s + w (d - s)."""
    q = tau * np.asarray(ninv, dtype=np.float64)
    return lam * q / (1.0 + (lam - 1.0) * q)


def harmonic_filter(cl, lam, tau, omega):
    """f_l(lambda) = C_l / (C_l + lambda tau Omega): Eq. (4) per harmonic mode."""
    cl = np.asarray(cl, dtype=np.float64)
    f = np.zeros_like(cl)
    pos = cl > 0
    f[pos] = cl[pos] / (cl[pos] + lam * tau * omega)
    return f


def expand_l(vals_l, lmax):
    """Broadcast a per-l array onto the packed alm layout."""
    out = np.empty(n_alm(lmax))
    for m in range(lmax + 1):
        i0 = alm_index(lmax, m, m)
        out[i0:i0 + lmax - m + 1] = vals_l[m:lmax + 1]
    return out


def sweep(s_map, d, ninv, cl, lam, tau, nside, lmax):
    """One messenger sweep at a given lambda; returns (new s map, new s alm)."""
    omega = healpix.pixel_area(nside)
    w = pixel_weight(ninv, lam, tau)
    t = s_map + w * (d - s_map)                               # Eq. (3)
    a = sht.map2alm(t, nside, lmax)                            # basis change
    s_alm = expand_l(harmonic_filter(cl, lam, tau, omega), lmax) * a   # Eq. (4)
    s_new = sht.alm2map(s_alm, nside, lmax)                    # back to pixels
    return s_new, s_alm


def solve(d, ninv, cl, lambdas, nside, lmax, callback=None):
    """Run the messenger iteration for the given lambda schedule (one sweep per
    entry), starting from s = t = 0. Returns (s_wf map, s_wf alm)."""
    ninv = np.asarray(ninv, dtype=np.float64)
    d = np.asarray(d, dtype=np.float64)
    tau = tau_of(ninv)
    s_map = np.zeros(healpix.npix(nside))
    s_alm = np.zeros(n_alm(lmax), dtype=np.complex128)
    for k, lam in enumerate(lambdas):
        s_map, s_alm = sweep(s_map, d, ninv, cl, float(lam), tau, nside, lmax)
        if callback is not None:
            callback(k, s_map, s_alm)
    return s_map, s_alm


def chi2(s_map, s_alm, d, ninv, cl, lmax, lam=1.0, tau=None):
    """chi^2_lambda(s) = s^dagger S^-1 s + (d - s)^dagger N_lambda^-1 (d - s).

    At lambda = 1 this is the paper's convergence monitor (Sect. 3).
    N_lambda = N + (lambda - 1) tau on observed pixels; S = diag(C_l) in the
    harmonic basis, modes with C_l = 0 excluded (they are zero in s).
    """
    ninv = np.asarray(ninv, dtype=np.float64)
    if tau is None:
        tau = tau_of(ninv)
    nl = ninv / (1.0 + (lam - 1.0) * tau * ninv)
    r = np.asarray(d) - np.asarray(s_map)
    cl = np.asarray(cl, dtype=np.float64)
    cinv = np.zeros_like(cl)
    cinv[cl > 0] = 1.0 / cl[cl > 0]
    prior = np.sum(sht.alm_weights(lmax) * expand_l(cinv, lmax) * np.abs(s_alm) ** 2)
    return float(prior + np.sum(nl * r * r))

