"""Spherical-harmonic transform pair on HEALPix rings (oracle; test infrastructure only).

The change of basis of the messenger iteration (Sect. 2: solve Eq. (3) in the
pixel basis, move to the basis where S is diagonal, solve Eq. (4), move back)
is, on the sphere, the spherical-harmonic transform pair:

  synthesis   f_p = sum_{l<=lmax} sum_{m=-l..l} a_lm Y_lm(theta_p, phi_p)
              = sum_l [ a_l0 lambda_l0(z_p)
                        + 2 Re sum_{m=1..l} a_lm lambda_lm(z_p) exp(i m phi_p) ]
              (real map: a_{l,-m} = (-1)^m conj(a_lm))
  analysis    a_lm = Omega sum_p conj(Y_lm(theta_p, phi_p)) f_p,  Omega = 4 pi / npix

The analysis is the pixel-area-weighted adjoint of the synthesis (no ring
weights, no iterative refinement): the reading adopted here for the transform
the paper leaves unspecified.

Both are split into a ring part (a discrete Fourier sum along each iso-latitude
ring) and a Legendre part (a sum over rings / over l for each m). The ring
sums are the plain definitions
  G_r(m) = sum_j f_j exp(-i m phi_j)            m = 0..lmax
  f_j    = sum_{m=-lmax..lmax} F_r(m) exp(i m phi_j),  F_r(-m) = conj(F_r(m))
evaluated with numpy's FFT as a library primitive: since phi_j = phi0 + 2 pi j /
n_phi, the sum over j at frequency m equals the length-n_phi DFT at bin
(m mod n_phi) times exp(-i m phi0), which also covers frequencies above the
ring's Nyquist bin (aliasing on short polar rings). `ring_analysis_direct` and
`ring_synthesis_direct` evaluate the same sums term by term for small inputs.
"""
import numpy as np

from . import healpix
from .legendre import lambda_m, sectoral, alm_index, n_alm


# ---------------------------------------------------------------- ring sums
def ring_analysis(maps, nside, lmax):
    """G[r, m] = sum_j f_{r,j} exp(-i m phi_{r,j}), m = 0..lmax (complex, no Omega)."""
    g = healpix.ring_info(nside)
    f = np.asarray(maps, dtype=np.float64)
    nr = len(g["z"])
    out = np.zeros((nr, lmax + 1), dtype=np.complex128)
    m = np.arange(lmax + 1)
    for r in range(nr):
        s, n = g["start"][r], g["nphi"][r]
        x = np.fft.fft(f[s:s + n])                       # sum_j f_j exp(-2 pi i k j / n)
        out[r] = x[m % n] * np.exp(-1j * m * g["phi0"][r])
    return out


def ring_synthesis(F, nside, lmax):
    """f_{r,j} = sum_{m=-lmax..lmax} F[r, |m|]^(*) exp(i m phi_{r,j}) for every ring."""
    g = healpix.ring_info(nside)
    F = np.asarray(F, dtype=np.complex128)
    out = np.zeros(healpix.npix(nside))
    m = np.arange(lmax + 1)
    for r in range(len(g["z"])):
        s, n = g["start"][r], g["nphi"][r]
        c = F[r] * np.exp(1j * m * g["phi0"][r])        # F(m) exp(i m phi0), m >= 0
        b = np.zeros(n, dtype=np.complex128)
        np.add.at(b, m % n, c)                           # m >= 0 terms into bin m mod n
        np.add.at(b, (-m[1:]) % n, np.conj(c[1:]))       # m < 0 terms: F(-m) = conj F(m)
        # f_j = sum_k b_k exp(+2 pi i k j / n) = n * ifft(b)
        out[s:s + n] = (np.fft.ifft(b) * n).real
    return out


def ring_analysis_direct(maps, nside, lmax):
    """Term-by-term version of ring_analysis (small inputs only)."""
    g = healpix.ring_info(nside)
    f = np.asarray(maps, dtype=np.float64)
    out = np.zeros((len(g["z"]), lmax + 1), dtype=np.complex128)
    for r in range(len(g["z"])):
        s, n = g["start"][r], g["nphi"][r]
        phi = g["phi0"][r] + 2.0 * np.pi * np.arange(n) / n
        for m in range(lmax + 1):
            out[r, m] = np.sum(f[s:s + n] * np.exp(-1j * m * phi))
    return out


def ring_synthesis_direct(F, nside, lmax):
    """Term-by-term version of ring_synthesis (small inputs only)."""
    g = healpix.ring_info(nside)
    out = np.zeros(healpix.npix(nside))
    for r in range(len(g["z"])):
        s, n = g["start"][r], g["nphi"][r]
        phi = g["phi0"][r] + 2.0 * np.pi * np.arange(n) / n
        acc = np.zeros(n, dtype=np.complex128)
        for m in range(-lmax, lmax + 1):
            c = F[r, m] if m >= 0 else np.conj(F[r, -m])
            acc += c * np.exp(1j * m * phi)
        out[s:s + n] = acc.real
    return out


# ---------------------------------------------------------------- SHT pair
def map2alm(maps, nside, lmax):
    """a_lm = Omega sum_p lambda_lm(z_p) exp(-i m phi_p) f_p (packed m-major, complex)."""
    g = healpix.ring_info(nside)
    G = ring_analysis(maps, nside, lmax)                  # [ring, m]
    omega = healpix.pixel_area(nside)
    seeds = sectoral(lmax, g["z"])
    alm = np.zeros(n_alm(lmax), dtype=np.complex128)
    for m in range(lmax + 1):
        lam = lambda_m(lmax, m, g["z"], seeds)           # [l-m, ring]
        i0 = alm_index(lmax, m, m)
        alm[i0:i0 + lmax - m + 1] = omega * (lam @ G[:, m])
    return alm


def alm2map(alm, nside, lmax):
    """f_p = sum_l sum_m a_lm Y_lm(p) for a real map (a_{l,-m} implied)."""
    g = healpix.ring_info(nside)
    alm = np.asarray(alm, dtype=np.complex128)
    seeds = sectoral(lmax, g["z"])
    F = np.zeros((len(g["z"]), lmax + 1), dtype=np.complex128)
    for m in range(lmax + 1):
        lam = lambda_m(lmax, m, g["z"], seeds)           # [l-m, ring]
        i0 = alm_index(lmax, m, m)
        F[:, m] = lam.T @ alm[i0:i0 + lmax - m + 1]
    return ring_synthesis(F, nside, lmax)


def map2alm_columns(maps, nside, lmax, ms):
    """The analysis restricted to a few m: {m: a_lm for l = m..lmax}, each from the
    same ring sums and Legendre values as map2alm (spot checks of large transforms,
    where the full Legendre sum over every m would take too long)."""
    g = healpix.ring_info(nside)
    G = ring_analysis(maps, nside, lmax)
    omega = healpix.pixel_area(nside)
    return {int(m): omega * (lambda_m(lmax, int(m), g["z"]) @ G[:, int(m)]) for m in ms}


def alm2map_columns(cols, nside, lmax):
    """Synthesis of a real field whose alm vanish outside the given m:
    cols = {m: a_lm for l = m..lmax}. Equals alm2map of the full packed array that
    holds these columns and zeros elsewhere."""
    g = healpix.ring_info(nside)
    F = np.zeros((len(g["z"]), lmax + 1), dtype=np.complex128)
    for m, a in cols.items():
        F[:, int(m)] = lambda_m(lmax, int(m), g["z"]).T @ np.asarray(a, dtype=np.complex128)
    return ring_synthesis(F, nside, lmax)


def alm_dot(a, b, lmax):
    """Real inner product of two real-field alm sets:
    sum_l [a_l0 b_l0 + 2 Re sum_{m>0} a_lm conj(b_lm)] (= sum over m=-l..l)."""
    w = np.full(n_alm(lmax), 2.0)
    w[:lmax + 1] = 1.0                                    # m = 0 block comes first
    return float(np.sum(w * (np.asarray(a) * np.conj(np.asarray(b))).real))


def alm_weights(lmax):
    """Real-degree-of-freedom weights per packed alm: 1 for m = 0, 2 for m > 0."""
    w = np.full(n_alm(lmax), 2.0)
    w[:lmax + 1] = 1.0
    return w


def alm_ell(lmax):
    """l of every packed alm entry."""
    out = np.empty(n_alm(lmax), dtype=np.int64)
    for m in range(lmax + 1):
        i0 = alm_index(lmax, m, m)
        out[i0:i0 + lmax - m + 1] = np.arange(m, lmax + 1)
    return out
