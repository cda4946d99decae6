"""Normalised associated Legendre functions (oracle; test infrastructure only).

The harmonic basis of the messenger iteration (Sect. 2: the signal covariance S
is diagonal in it) is the spherical harmonics Y_lm(theta, phi) =
lambda_lm(cos theta) exp(i m phi) with

  lambda_lm(z) = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!) P_l^m(z)

including the Condon-Shortley phase (-1)^m in P_l^m. This is the textbook
definition; the paper itself does not fix a convention.

Computed by the standard three-term recurrences (written from the definition):
  sectoral seed  lambda_00 = 1/sqrt(4 pi),
                 lambda_mm = -sqrt((2m+1)/(2m)) sin(theta) lambda_{m-1,m-1}
  first step     lambda_{m+1,m} = sqrt(2m+3) z lambda_mm
  l-recurrence   lambda_lm = a_lm (z lambda_{l-1,m} - lambda_{l-2,m} / a_{l-1,m}),
                 a_lm = sqrt((4 l^2 - 1) / (l^2 - m^2)).

lambda_mm underflows double precision near the poles for large m, while the
l-recurrence can grow it back to O(1). The oracle therefore carries every value
as (mantissa, binary exponent) until the exponent returns to zero; values that
stay below the double range come out as (exactly or nearly) zero.
"""
import numpy as np

_RESCALE_LOG2 = 100  # rescale when the mantissa exceeds 2**100


def sectoral(mmax, z):
    """Sectoral seeds lambda_mm(z) for m = 0..mmax as (mantissa, exponent).

    Returns (mant, expo) with shapes [mmax+1, len(z)]; lambda_mm = mant * 2**expo.
    """
    z = np.atleast_1d(np.asarray(z, dtype=np.float64))
    sin_t = np.sqrt((1.0 - z) * (1.0 + z))
    mant = np.empty((mmax + 1, z.size))
    expo = np.zeros((mmax + 1, z.size), dtype=np.int64)
    cur = np.full(z.size, 1.0 / np.sqrt(4.0 * np.pi))
    cur_e = np.zeros(z.size, dtype=np.int64)
    mant[0], expo[0] = cur, cur_e
    for m in range(1, mmax + 1):
        cur = -np.sqrt((2.0 * m + 1.0) / (2.0 * m)) * sin_t * cur
        f, e = np.frexp(cur)          # renormalise so the mantissa never underflows
        cur, cur_e = f, cur_e + e
        mant[m], expo[m] = cur, cur_e
    return mant, expo


def lambda_m(lmax, m, z, seeds=None):
    """lambda_lm(z) for l = m..lmax, one fixed m. Shape [lmax-m+1, len(z)].

    `seeds` may carry the output of `sectoral` (to avoid recomputing it)."""
    z = np.atleast_1d(np.asarray(z, dtype=np.float64))
    if seeds is None:
        seeds = sectoral(m, z)
    mant, expo = seeds
    nl = lmax - m + 1
    out = np.zeros((nl, z.size))
    if nl <= 0:
        return out
    v2 = mant[m].copy()                   # lambda_{l-2}, scaled
    e = expo[m].copy()                    # common exponent of v1, v2 (<= 0 or small)
    out[0] = np.ldexp(v2, e.astype(np.int32))
    if nl == 1:
        return out
    a_prev = np.sqrt(2.0 * m + 3.0)
    v1 = a_prev * z * v2                  # lambda_{m+1,m}
    out[1] = np.ldexp(v1, e.astype(np.int32))
    for l in range(m + 2, lmax + 1):
        a = np.sqrt((4.0 * l * l - 1.0) / ((l - m) * (l + m)))
        v = a * (z * v1 - v2 / a_prev)
        v2, v1, a_prev = v1, v, a
        # bring the exponent back towards zero while the value grows
        big = (e < 0) & (np.abs(v1) > 2.0 ** _RESCALE_LOG2)
        if big.any():
            k = np.minimum(-e[big], _RESCALE_LOG2)
            v1[big] = np.ldexp(v1[big], -k.astype(np.int32))
            v2[big] = np.ldexp(v2[big], -k.astype(np.int32))
            e[big] += k
        out[l - m] = np.ldexp(v1, e.astype(np.int32))
    return out


def lambda_all(lmax, z):
    """All lambda_lm(z) for 0 <= m <= l <= lmax in HEALPix packed order.

    Shape [N_lm, len(z)], row index m*(2*lmax+1-m)//2 + l."""
    z = np.atleast_1d(np.asarray(z, dtype=np.float64))
    seeds = sectoral(lmax, z)
    nlm = (lmax + 1) * (lmax + 2) // 2
    out = np.empty((nlm, z.size))
    for m in range(lmax + 1):
        i0 = m * (2 * lmax + 1 - m) // 2 + m
        out[i0:i0 + lmax - m + 1] = lambda_m(lmax, m, z, seeds)
    return out


def alm_index(lmax, l, m):
    """Packed m-major index of (l, m): m*(2*lmax+1-m)/2 + l (HEALPix order)."""
    return m * (2 * lmax + 1 - m) // 2 + l


def n_alm(lmax):
    return (lmax + 1) * (lmax + 2) // 2
