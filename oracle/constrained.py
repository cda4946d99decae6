"""Constrained realisations (oracle; test infrastructure only).

Elsner & Wandelt, Sect. 3 (power-spectrum figure): a constrained realisation is
the Wiener-filter map plus a fluctuation map; its power spectrum is unbiased
with respect to the fiducial spectrum.

Reading adopted where the paper is silent on how the fluctuation map is made
(listed in the design notes): the construction of Hoffman & Ribak (1991). With
a signal draw s_rand from N(0, S) and a noise draw n_rand from N(0, N),

    s_CR = WF(d) + [s_rand - WF(s_rand + n_rand)] = s_rand + WF(d - s_rand - n_rand)

(the Wiener filter is linear in the data), i.e. one solve with a modified data
map. The draws are built from unit normal draws passed in by the caller:
s_rand = alm2map(sqrt(C_l) xi) (xi_l0 real) and n_rand_p = eta_p / sqrt(N^-1_p),
zero where the pixel is unobserved (infinite noise, zero weight in every step).
"""
import numpy as np

from . import messenger, sht
from .legendre import alm_index


def signal_draw_alm(cl, xi, lmax):
    """sqrt(C_l) xi on the packed alm, real at m = 0."""
    cl = np.asarray(cl, dtype=np.float64)
    out = np.array(xi, dtype=np.complex128)
    for m in range(lmax + 1):
        i0, i1 = alm_index(lmax, m, m), alm_index(lmax, lmax, m) + 1
        out[i0:i1] = np.sqrt(cl[m:lmax + 1]) * (out[i0:i1].real if m == 0 else out[i0:i1])
    return out


def noise_draw(ninv, eta):
    """eta / sqrt(N^-1), 0 where N^-1 = 0."""
    ninv = np.asarray(ninv, dtype=np.float64)
    out = np.zeros_like(ninv)
    obs = ninv > 0
    out[obs] = np.asarray(eta, dtype=np.float64)[obs] / np.sqrt(ninv[obs])
    return out


def constrained(d, ninv, cl, xi, eta, nside, lmax, wf):
    """s_CR and its alm for a Wiener filter wf: data map -> (map, alm)."""
    a_rand = signal_draw_alm(cl, xi, lmax)
    s_rand = sht.alm2map(a_rand, nside, lmax)
    s_wf, a_wf = wf(np.asarray(d, dtype=np.float64) - s_rand - noise_draw(ninv, eta))
    return s_rand + s_wf, a_rand + a_wf


def constrained_messenger(d, ninv, cl, xi, eta, lambdas, nside, lmax):
    """The same with the messenger solve of a fixed lambda schedule as the filter."""
    return constrained(d, ninv, cl, xi, eta, nside, lmax,
                       lambda x: messenger.solve(x, ninv, cl, lambdas, nside, lmax))
