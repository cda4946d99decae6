"""Shared helpers of the test suite (input construction and error metrics)."""
import numpy as np

from oracle import healpix, sht
from paper_1211_0585_amd import synth


def rel_l2(x, ref, w=None):
    x = np.asarray(x)
    ref = np.asarray(ref)
    if w is None:
        return float(np.linalg.norm((x - ref).ravel()) / max(np.linalg.norm(ref.ravel()), 1e-300))
    num = np.sqrt(np.sum(w * np.abs(x - ref) ** 2))
    den = np.sqrt(np.sum(w * np.abs(ref) ** 2))
    return float(num / max(den, 1e-300))


def alm_rel_l2(x, ref, lmax):
    """Relative L2 over real degrees of freedom (weight 1 for m = 0, 2 for m > 0)."""
    return rel_l2(x, ref, sht.alm_weights(lmax))


def small_band_inputs(nside, lmax, seed=0):
    """Nside-16-style recipe at any size; d = oracle synthesis of the drawn alm + noise."""
    theta, _ = healpix.pixel_angles(nside)
    c = synth.small_band_case(theta, lmax, seed=seed)
    c["d"] = sht.alm2map(c["signal_alm"], nside, lmax) + c["noise"]
    return c


def satellite_inputs(nside, lmax, seed=0, **kw):
    theta, phi = healpix.pixel_angles(nside)
    c = synth.satellite_case(theta, phi, lmax, seed=seed, **kw)
    c["d"] = sht.alm2map(c["signal_alm"], nside, lmax) + c["noise"]
    return c


def random_alm(lmax, seed):
    rs = np.random.default_rng(seed)
    n = (lmax + 1) * (lmax + 2) // 2
    a = rs.standard_normal(n) + 1j * rs.standard_normal(n)
    a[:lmax + 1] = a[:lmax + 1].real
    return a
