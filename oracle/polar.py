"""Polarised (T, Q, U) messenger Wiener filter (oracle; test infrastructure only).

The paper filters temperature and polarisation maps together (Sect. 3: the WMAP
temperature and polarisation data with their T and P masks; Sect. 4: the method
stays robust with polarisation included). Eqs. (3)-(4) then hold per pixel for a
3-vector (T, Q, U) with a 3x3 noise covariance N_p, and per harmonic mode for a
3-vector (T, E, B) with the 3x3 signal covariance C_l of the TT, EE, BB and TE
spectra (TB = EB = 0). The paper gives no formulas for the polarised transform;
this module writes out the textbook ones (readings P1-P6 of the design notes):

P1 Spin-weighted harmonics sY_lm(theta, phi) = s_lambda_lm(theta) exp(i m phi),
   defined by Goldberg et al. (1967, J. Math. Phys. 8, 2155), Eq. (3.1) there:
     sY_lm = (-1)^m sqrt((l+m)!(l-m)!(2l+1) / (4 pi (l+s)!(l-s)!)) sin^{2l}(theta/2)
             sum_r C(l-s, r) C(l+s, r+s-m) (-1)^{l-r-s} exp(i m phi) cot^{2r+s-m}(theta/2)
   At s = 0 this is Y_lm with the Condon-Shortley phase (the spin-0 basis).
   Polarisation: Q +/- iU = sum_lm a_{+/-2,lm} (+/-2)Y_lm, a_{+/-2} = -(a_E +/- i a_B)
   (Zaldarriaga & Seljak 1997). With lambda+ = (2lam + (-2)lam)/2 and
   lambda- = (2lam - (-2)lam)/2, and a_{l,-m} = (-1)^m conj(a_lm) for E and B,
     Q = sum_{m=-l..l} [-E lambda+ - i B lambda-] e^{i m phi},
     U = sum_{m=-l..l} [-B lambda+ + i E lambda-] e^{i m phi},
   a real-field ring synthesis of the m >= 0 coefficients, as for T.
P2 Analysis = Omega-weighted adjoint: a_{+/-2,lm} = Omega sum_p (Q +/- iU)_p conj((+/-2)Y_lm(p)),
   a_E = -(a_2 + a_-2)/2, a_B = i (a_2 - a_-2)/2, i.e.
     E_lm = -sum_p [lambda+ Q_p + i lambda- U_p] Omega e^{-i m phi_p},
     B_lm =  sum_p [-lambda+ U_p + i lambda- Q_p] Omega e^{-i m phi_p};  a_T as for spin 0.
P3 tau = min over pixels of the smallest eigenvalue of N_p = 1 / max_p lambda_max(N^-1_p):
   the largest T = tau 1 with Nbar = N - T positive semi-definite (for a diagonal N
   this is the paper's min(diag N)).
P4 Eq. (3) per pixel: t = s + W (d - s), W = lambda tau M (1 + (lambda - 1) M)^-1 with
   M = tau N^-1_p (3x3), the form of (Nbar^-1 + (lambda T)^-1) t = Nbar^-1 d + (lambda T)^-1 s
   without inverting Nbar (singular at the least-noisy pixel, infinite where masked).
P5 Eq. (4) per (l, m): s = F_l a, F_l = C_l (C_l + lambda tau Omega 1)^-1 (3x3 with the TE
   coupling; E and B have no l < 2 modes, so F is 0 there for them).
P6 Masks: bit 0 of a pixel's mask byte = T observed, bit 1 = Q/U observed; an unobserved
   component has its rows and columns of N^-1 set to zero.

Maps are arrays [3, npix] (T, Q, U), alm arrays [3, N_lm] (T, E, B) in the packed
m-major order of the spin-0 transforms. The noise precision is given per pixel as
six arrays [6, npix]: the TT, QQ, UU, TQ, TU, QU entries of N^-1_p.
"""
import numpy as np
from math import comb, factorial, pi

from . import healpix, sht
from .legendre import alm_index, n_alm

NINV_ORDER = ("TT", "QQ", "UU", "TQ", "TU", "QU")


# ---------------------------------------------------------------- spin-weighted functions
def goldberg(l, m, s, theta):
    """s_lambda_lm(theta) from Goldberg et al.'s explicit sum (P1), in float64.

    Direct evaluation for small l (the sum cancels heavily at large l); any
    integer m and s with |m|, |s| <= l, else 0."""
    theta = np.asarray(theta, dtype=np.float64)
    if l < abs(s) or l < abs(m):
        return np.zeros_like(theta)
    pre = (-1) ** m * np.sqrt(factorial(l + m) * factorial(l - m) * (2 * l + 1)
                              / (4.0 * pi * factorial(l + s) * factorial(l - s)))
    sh, ch = np.sin(0.5 * theta), np.cos(0.5 * theta)
    tot = np.zeros_like(theta)
    for r in range(l - s + 1):
        k = r + s - m
        if k < 0 or k > l + s:
            continue
        e = 2 * r + s - m                     # cot^e(theta/2) sin^{2l}(theta/2)
        tot = tot + comb(l - s, r) * comb(l + s, k) * (-1) ** (l - r - s) * ch ** e * sh ** (2 * l - e)
    return pre * tot


def spin_sectoral(mmax, s, z):
    """Seeds s_lambda at l0 = max(m, |s|) for m = 0..mmax as (mantissa, exponent)
    arrays [mmax+1, len(z)] (s = +2 or -2; t = theta).

    From the one surviving term of Goldberg's sum (P1):
      m <  |s| (l0 = |s|):
          s > 0: (-1)^m sqrt((2s+1)/(4 pi) (2s)!/((s+m)!(s-m)!)) sin^{s+m}(t/2) cos^{s-m}(t/2)
          s < 0: (-1)^s sqrt((2|s|+1)/(4 pi) (2|s|)!/((|s|+m)!(|s|-m)!)) sin^{|s|-m}(t/2) cos^{|s|+m}(t/2)
      m >= |s| (l0 = m):
          (-1)^m sqrt((2m+1)(2m)! / (4 pi (m+s)!(m-s)!)) sin^{m+s}(t/2) cos^{m-s}(t/2),
    the last built up from its value at m = |s|, (-1)^|s| sqrt((2|s|+1)/(4 pi)) times
    sin^{2|s|}(t/2) (s > 0) or cos^{2|s|}(t/2) (s < 0), by the ratio of consecutive m,
          value(m+1) / value(m) = -sqrt((2m+3)(2m+2) / ((m+1+s)(m+1-s))) sin(t/2) cos(t/2),
    with the mantissa renormalised at every step."""
    z = np.atleast_1d(np.asarray(z, dtype=np.float64))
    a = abs(s)
    sh = np.sqrt(0.5 * (1.0 - z))
    ch = np.sqrt(0.5 * (1.0 + z))
    mant = np.zeros((mmax + 1, z.size))
    expo = np.zeros((mmax + 1, z.size), dtype=np.int64)
    for m in range(min(a, mmax + 1)):
        if s > 0:
            v = ((-1) ** m * np.sqrt((2 * a + 1) / (4 * pi) * factorial(2 * a) / (factorial(a + m) * factorial(a - m)))
                 * sh ** (a + m) * ch ** (a - m))
        else:
            v = ((-1) ** a * np.sqrt((2 * a + 1) / (4 * pi) * factorial(2 * a) / (factorial(a + m) * factorial(a - m)))
                 * sh ** (a - m) * ch ** (a + m))
        mant[m], expo[m] = np.frexp(v)
    if mmax < a:
        return mant, expo
    cur = (-1) ** a * np.sqrt((2 * a + 1) / (4 * pi)) * (sh if s > 0 else ch) ** (2 * a)
    cur, e = np.frexp(cur)
    e = e.astype(np.int64)
    mant[a], expo[a] = cur, e
    for m in range(a, mmax):
        r = -np.sqrt((2.0 * m + 3.0) * (2.0 * m + 2.0) / ((m + 1.0 + s) * (m + 1.0 - s)))
        cur, de = np.frexp(r * sh * ch * cur)
        e = e + de
        mant[m + 1], expo[m + 1] = cur, e
    return mant, expo


def spin_lambda_m(lmax, m, s, z, seeds=None):
    """s_lambda_lm(z) for l = m..lmax at one m >= 0, shape [lmax-m+1, len(z)]; rows
    with l < |s| are zero. Three-term recurrence of the Wigner d-functions
    (Edmonds 1957, Eq. 4.1.x; written for the normalised s_lambda):
      y_{l+1} = (a_l z + b_l) y_l - c_l y_{l-1},   K_l = sqrt(((l+1)^2 - m^2)((l+1)^2 - s^2))
      a_l = sqrt((2l+3)(2l+1)) (l+1) / K_l,  b_l = sqrt((2l+3)(2l+1)) m s / (l K_l),
      c_l = (l+1)/l sqrt((2l+3)/(2l-1)) sqrt((l^2-m^2)(l^2-s^2)) / K_l,
    started at l0 = max(m, |s|) from `spin_sectoral` (y_{l0-1} = 0). At s = 0 it is
    the spin-0 recurrence. Values are carried as (mantissa, exponent) until the
    exponent returns to zero, as in the spin-0 functions."""
    z = np.atleast_1d(np.asarray(z, dtype=np.float64))
    nl = lmax - m + 1
    out = np.zeros((max(nl, 0), z.size))
    l0 = max(m, abs(s))
    if l0 > lmax:
        return out
    if seeds is None:
        seeds = spin_sectoral(m, s, z)
    y1 = seeds[0][m].copy()          # y_l
    e = seeds[1][m].copy()
    y0 = np.zeros_like(y1)           # y_{l-1}
    out[l0 - m] = np.ldexp(y1, e.astype(np.int32))
    for l in range(l0, lmax):
        K = np.sqrt(((l + 1) ** 2 - m * m) * ((l + 1) ** 2 - s * s))
        a = np.sqrt((2 * l + 3) * (2 * l + 1)) * (l + 1) / K
        b = np.sqrt((2 * l + 3) * (2 * l + 1)) * m * s / (l * K)
        c = (l + 1) / l * np.sqrt((2 * l + 3) / (2 * l - 1)) * np.sqrt((l * l - m * m) * (l * l - s * s)) / K
        y = (a * z + b) * y1 - c * y0
        y0, y1 = y1, y
        big = (e < 0) & (np.abs(y1) > 2.0 ** 100)
        if big.any():
            k = np.minimum(-e[big], 100)
            y1[big] = np.ldexp(y1[big], -k.astype(np.int32))
            y0[big] = np.ldexp(y0[big], -k.astype(np.int32))
            e[big] += k
        out[l + 1 - m] = np.ldexp(y1, e.astype(np.int32))
    return out


def lambda_pm(lmax, m, z, seeds=None):
    """(lambda+, lambda-) = ((2)lam + (-2)lam)/2, ((2)lam - (-2)lam)/2 for l = m..lmax;
    `seeds` may carry (spin_sectoral(., 2, z), spin_sectoral(., -2, z))."""
    if seeds is None:
        seeds = (spin_sectoral(m, 2, z), spin_sectoral(m, -2, z))
    p = spin_lambda_m(lmax, m, 2, z, seeds[0])
    q = spin_lambda_m(lmax, m, -2, z, seeds[1])
    return 0.5 * (p + q), 0.5 * (p - q)


# ---------------------------------------------------------------- polarised SHT pair
def map2alm(maps, nside, lmax):
    """[T, Q, U] maps -> [T, E, B] packed alm (P2): Omega-weighted adjoint of alm2map."""
    maps = np.asarray(maps, dtype=np.float64)
    g = healpix.ring_info(nside)
    omega = healpix.pixel_area(nside)
    out = np.zeros((3, n_alm(lmax)), dtype=np.complex128)
    out[0] = sht.map2alm(maps[0], nside, lmax)
    GQ = omega * sht.ring_analysis(maps[1], nside, lmax)
    GU = omega * sht.ring_analysis(maps[2], nside, lmax)
    seeds = (spin_sectoral(lmax, 2, g["z"]), spin_sectoral(lmax, -2, g["z"]))
    for m in range(lmax + 1):
        lp, lm = lambda_pm(lmax, m, g["z"], seeds)
        i0 = alm_index(lmax, m, m)
        sl = slice(i0, i0 + lmax - m + 1)
        out[1, sl] = -(lp @ GQ[:, m] + 1j * (lm @ GU[:, m]))
        out[2, sl] = -(lp @ GU[:, m]) + 1j * (lm @ GQ[:, m])
    return out


def alm2map(alm, nside, lmax):
    """[T, E, B] packed alm -> [T, Q, U] maps (P1). The imaginary parts of the m = 0
    coefficients are ignored (real fields)."""
    alm = np.array(alm, dtype=np.complex128)
    alm[:, :lmax + 1] = alm[:, :lmax + 1].real
    g = healpix.ring_info(nside)
    out = np.zeros((3, healpix.npix(nside)))
    out[0] = sht.alm2map(alm[0], nside, lmax)
    FQ = np.zeros((len(g["z"]), lmax + 1), dtype=np.complex128)
    FU = np.zeros_like(FQ)
    seeds = (spin_sectoral(lmax, 2, g["z"]), spin_sectoral(lmax, -2, g["z"]))
    for m in range(lmax + 1):
        lp, lm = lambda_pm(lmax, m, g["z"], seeds)
        i0 = alm_index(lmax, m, m)
        e = alm[1, i0:i0 + lmax - m + 1]
        b = alm[2, i0:i0 + lmax - m + 1]
        FQ[:, m] = lp.T @ (-e) + lm.T @ (-1j * b)
        FU[:, m] = lp.T @ (-b) + lm.T @ (1j * e)
    out[1] = sht.ring_synthesis(FQ, nside, lmax)
    out[2] = sht.ring_synthesis(FU, nside, lmax)
    return out


def _all_m_coeffs(alm_row, lmax, sign_neg):
    """{(l, m): coefficient} for m = -l..l of a real field's packed alm."""
    out = {}
    for m in range(lmax + 1):
        for l in range(m, lmax + 1):
            a = alm_row[alm_index(lmax, l, m)]
            out[(l, m)] = a
            if m > 0:
                out[(l, -m)] = (-1) ** m * np.conj(a)
    return out


def alm2map_direct(alm, nside, lmax):
    """alm2map by the defining sums at every pixel (small inputs only): T from the
    spin-0 Y_lm, Q +/- iU = sum over m = -l..l of a_{+/-2,lm} (+/-2)Y_lm with Goldberg's
    functions, a_{+/-2} = -(E +/- iB) and E, B extended to m < 0 as real fields."""
    alm = np.array(alm, dtype=np.complex128)
    alm[:, :lmax + 1] = alm[:, :lmax + 1].real
    theta, phi = healpix.pixel_angles(nside)
    T = _all_m_coeffs(alm[0], lmax, None)
    E = _all_m_coeffs(alm[1], lmax, None)
    B = _all_m_coeffs(alm[2], lmax, None)
    t = np.zeros(theta.size, dtype=np.complex128)
    p2 = np.zeros_like(t)
    m2 = np.zeros_like(t)
    for (l, m), aT in T.items():
        ph = np.exp(1j * m * phi)
        t += aT * goldberg(l, m, 0, theta) * ph
        if l >= 2:
            p2 += -(E[(l, m)] + 1j * B[(l, m)]) * goldberg(l, m, 2, theta) * ph
            m2 += -(E[(l, m)] - 1j * B[(l, m)]) * goldberg(l, m, -2, theta) * ph
    return np.stack([t.real, 0.5 * (p2 + m2).real, (0.5 / 1j * (p2 - m2)).real])


def map2alm_direct(maps, nside, lmax):
    """map2alm by the defining sums (small inputs only): a_T = Omega sum conj(Y) T,
    a_{+/-2} = Omega sum (Q +/- iU) conj((+/-2)Y), E = -(a_2 + a_-2)/2, B = i(a_2 - a_-2)/2."""
    maps = np.asarray(maps, dtype=np.float64)
    theta, phi = healpix.pixel_angles(nside)
    omega = healpix.pixel_area(nside)
    out = np.zeros((3, n_alm(lmax)), dtype=np.complex128)
    qp = maps[1] + 1j * maps[2]
    qm = maps[1] - 1j * maps[2]
    for m in range(lmax + 1):
        ph = np.exp(-1j * m * phi)
        for l in range(m, lmax + 1):
            i = alm_index(lmax, l, m)
            out[0, i] = omega * np.sum(maps[0] * goldberg(l, m, 0, theta) * ph)
            if l >= 2:
                a2 = omega * np.sum(qp * goldberg(l, m, 2, theta) * ph)
                am2 = omega * np.sum(qm * goldberg(l, m, -2, theta) * ph)
                out[1, i] = -0.5 * (a2 + am2)
                out[2, i] = 0.5j * (a2 - am2)
    return out


def alm_dot(a, b, lmax):
    """Real inner product of two [T, E, B] alm sets (sum of the spin-0 inner products)."""
    return sum(sht.alm_dot(a[f], b[f], lmax) for f in range(3))


# ---------------------------------------------------------------- noise and signal models
def ninv_matrices(ninv6, mask=None):
    """[npix, 3, 3] N^-1_p from the six [6, npix] entries (P6 applied with `mask`)."""
    n6 = np.asarray(ninv6, dtype=np.float64)
    tt, qq, uu, tq, tu, qu = n6
    M = np.empty((n6.shape[1], 3, 3))
    M[:, 0, 0], M[:, 1, 1], M[:, 2, 2] = tt, qq, uu
    M[:, 0, 1] = M[:, 1, 0] = tq
    M[:, 0, 2] = M[:, 2, 0] = tu
    M[:, 1, 2] = M[:, 2, 1] = qu
    if mask is not None:
        mask = np.asarray(mask, dtype=np.uint8)
        keep = np.stack([(mask & 1) != 0, (mask & 2) != 0, (mask & 2) != 0], axis=1).astype(np.float64)
        M = M * keep[:, :, None] * keep[:, None, :]
    return M


def tau_of(M):
    """P3: tau = 1 / max_p lambda_max(N^-1_p)."""
    lmx = np.linalg.eigvalsh(M)[:, -1].max()
    if not lmx > 0:
        raise ValueError("no observed pixel")
    return 1.0 / lmx


def pixel_update(s, d, M, lam, tau):
    """Eq. (3) per pixel (P4): t = s + lambda tau M (1 + (lambda-1) tau M)^-1 (d - s),
    with M = N^-1_p; s, d of shape [3, npix]."""
    q = tau * M
    A = np.eye(3)[None] + (lam - 1.0) * q
    r = (np.asarray(d) - np.asarray(s)).T                      # [npix, 3]
    v = np.einsum("pij,pj->pi", q, r)
    y = np.linalg.solve(A, v[:, :, None])[:, :, 0]
    return np.asarray(s) + lam * y.T


def cl_matrices(cl4):
    """[lmax+1, 3, 3] C_l from the four spectra [TT, EE, BB, TE] (TB = EB = 0)."""
    tt, ee, bb, te = np.asarray(cl4, dtype=np.float64)
    C = np.zeros((tt.size, 3, 3))
    C[:, 0, 0], C[:, 1, 1], C[:, 2, 2] = tt, ee, bb
    C[:, 0, 1] = C[:, 1, 0] = te
    return C


def harmonic_filter(cl4, lam, tau, omega):
    """Eq. (4) per mode (P5): F_l = C_l (C_l + lambda tau Omega 1)^-1, [lmax+1, 3, 3]."""
    C = cl_matrices(cl4)
    mu = lam * tau * omega
    F = np.empty_like(C)
    for l in range(C.shape[0]):
        F[l] = C[l] @ np.linalg.inv(C[l] + mu * np.eye(3))
    F[:2, 1:, :] = 0.0          # no E, B modes below l = 2
    F[:2, :, 1:] = 0.0
    return F


def apply_filter(F, alm, lmax):
    """s_lm = F_l a_lm for [3, N_lm] alm."""
    ell = sht.alm_ell(lmax)
    return np.einsum("kij,jk->ik", F[ell], alm)


# ---------------------------------------------------------------- the iteration
def sweep(s_map, d, M, cl4, lam, tau, nside, lmax):
    """One polarised messenger sweep: Eq. (3), analysis, Eq. (4), synthesis."""
    t = pixel_update(s_map, d, M, lam, tau)
    a = map2alm(t, nside, lmax)
    s_alm = apply_filter(harmonic_filter(cl4, lam, tau, healpix.pixel_area(nside)), a, lmax)
    return alm2map(s_alm, nside, lmax), s_alm


def solve(d, ninv6, cl4, lambdas, nside, lmax, mask=None, callback=None):
    """Messenger iteration from s = t = 0, one sweep per lambda. Returns
    (s_wf maps [3, npix], s_wf alm [3, N_lm])."""
    M = ninv_matrices(ninv6, mask)
    tau = tau_of(M)
    s_map = np.zeros((3, healpix.npix(nside)))
    s_alm = np.zeros((3, n_alm(lmax)), dtype=np.complex128)
    for k, lam in enumerate(lambdas):
        s_map, s_alm = sweep(s_map, np.asarray(d, dtype=np.float64), M, cl4, float(lam), tau, nside, lmax)
        if callback is not None:
            callback(k, s_map, s_alm)
    return s_map, s_alm


def chi2(s_map, s_alm, d, M, cl4, lmax, lam=1.0, tau=None):
    """chi^2_lambda(s) = sum_lm w_m a^dagger C_l^+ a + sum_p r^T N_lambda,p^-1 r, r = d - s,
    N_lambda^-1 = N^-1 (1 + (lambda-1) tau N^-1)^-1, C^+ the pseudo-inverse (modes with
    no signal power carry none of s)."""
    if tau is None:
        tau = tau_of(M)
    C = cl_matrices(cl4)
    Cp = np.stack([np.linalg.pinv(C[l]) for l in range(C.shape[0])])
    ell = sht.alm_ell(lmax)
    w = sht.alm_weights(lmax)
    a = np.asarray(s_alm)
    prior = np.real(np.einsum("k,ik,kij,jk->", w, np.conj(a), Cp[ell], a))
    r = (np.asarray(d) - np.asarray(s_map)).T
    Nl = np.linalg.solve(np.eye(3)[None] + (lam - 1.0) * tau * M, M)
    data = np.einsum("pi,pij,pj->", r, Nl, r)
    return float(prior + data)


# ---------------------------------------------------------------- dense solves (tiny Nside)
def real_modes(cl4, lmax):
    """Real orthonormal basis of the polarised fields: (field, l, m, kind) with field
    0 = T, 1 = E, 2 = B, kind 0 = m=0, 1 = cos, 2 = sin (as in the spin-0 dense
    solves), for the fields with positive power at that l (E and B from l = 2)."""
    C = cl_matrices(cl4)
    out = []
    for l in range(lmax + 1):
        for f in range(3):
            if (f > 0 and l < 2) or not C[l, f, f] > 0:
                continue
            out.append((f, l, 0, 0))
            for m in range(1, l + 1):
                out.append((f, l, m, 1))
                out.append((f, l, m, 2))
    return out


def x_to_alm(x, modes, lmax):
    """Real-basis coefficients -> [3, N_lm] packed alm (a_lm = (x^c - i x^s)/sqrt 2)."""
    alm = np.zeros((3, n_alm(lmax)), dtype=np.complex128)
    for k, (f, l, m, kind) in enumerate(modes):
        i = alm_index(lmax, l, m)
        if kind == 0:
            alm[f, i] += x[k]
        elif kind == 1:
            alm[f, i] += x[k] / np.sqrt(2.0)
        else:
            alm[f, i] += -1j * x[k] / np.sqrt(2.0)
    return alm


def synthesis_matrix(modes, nside, lmax):
    """Y[(field, pixel), k]: the [3 npix] map of real basis function k."""
    npx = healpix.npix(nside)
    Y = np.empty((3 * npx, len(modes)))
    for k in range(len(modes)):
        e = np.zeros(len(modes))
        e[k] = 1.0
        Y[:, k] = alm2map(x_to_alm(e, modes, lmax), nside, lmax).reshape(-1)
    return Y


def _mode_cov(modes, cl4):
    """Signal covariance in the real basis: C_l[f, f'] between modes of the same (l, m, kind)."""
    C = cl_matrices(cl4)
    n = len(modes)
    S = np.zeros((n, n))
    for i, (f, l, m, k) in enumerate(modes):
        for j, (g, l2, m2, k2) in enumerate(modes):
            if (l, m, k) == (l2, m2, k2):
                S[i, j] = C[l, f, g]
    return S


def _block_pixels(Mp):
    """[3 npix, 3 npix] matrix of per-pixel 3x3 blocks Mp [npix, 3, 3] in (field, pixel) order."""
    npx = Mp.shape[0]
    out = np.zeros((3 * npx, 3 * npx))
    idx = np.arange(npx)
    for a in range(3):
        for b in range(3):
            out[a * npx + idx, b * npx + idx] = Mp[:, a, b]
    return out


def wiener_dense(d, ninv6, cl4, nside, lmax, mask=None):
    """Eq. (2) for the polarised fields: [C^-1 + Y^T N^-1 Y] x = Y^T N^-1 d. Returns (maps, alm)."""
    modes = real_modes(cl4, lmax)
    Y = synthesis_matrix(modes, nside, lmax)
    Nb = _block_pixels(ninv_matrices(ninv6, mask))
    A = np.linalg.inv(_mode_cov(modes, cl4)) + Y.T @ Nb @ Y
    x = np.linalg.solve(A, Y.T @ Nb @ np.asarray(d, dtype=np.float64).reshape(-1))
    return (Y @ x).reshape(3, -1), x_to_alm(x, modes, lmax)


def messenger_fixed_point(d, ninv6, cl4, lam, nside, lmax, mask=None):
    """Fixed point of the polarised sweep at a fixed lambda (the spin-0 derivation with
    3x3 blocks: F^-1 = 1 + lambda tau Omega C^-1 and W / (lambda tau) = N_lambda^-1):
      [C^-1 + Y^T N_l^-1 Y + (lambda tau Omega)^-1 (1 - Omega Y^T Y)] x = Y^T N_l^-1 d,
      N_l^-1 = N^-1 (1 + (lambda - 1) tau N^-1)^-1 per pixel."""
    modes = real_modes(cl4, lmax)
    Y = synthesis_matrix(modes, nside, lmax)
    M = ninv_matrices(ninv6, mask)
    tau = tau_of(M)
    omega = healpix.pixel_area(nside)
    Nl = np.linalg.solve(np.eye(3)[None] + (lam - 1.0) * tau * M, M)
    Nb = _block_pixels(Nl)
    n = len(modes)
    A = (np.linalg.inv(_mode_cov(modes, cl4)) + Y.T @ Nb @ Y
         + (np.eye(n) - omega * (Y.T @ Y)) / (lam * tau * omega))
    x = np.linalg.solve(A, Y.T @ Nb @ np.asarray(d, dtype=np.float64).reshape(-1))
    return (Y @ x).reshape(3, -1), x_to_alm(x, modes, lmax)


def iteration_matrix(ninv6, cl4, lam, nside, lmax, mask=None):
    """x_{k+1} = G x_k + const for one sweep in the real basis: G = F Omega Y^T (1 - W) Y."""
    modes = real_modes(cl4, lmax)
    Y = synthesis_matrix(modes, nside, lmax)
    M = ninv_matrices(ninv6, mask)
    tau = tau_of(M)
    omega = healpix.pixel_area(nside)
    q = tau * M
    W = lam * np.linalg.solve(np.eye(3)[None] + (lam - 1.0) * q, q)
    Ib = np.eye(3 * M.shape[0]) - _block_pixels(W)
    S = _mode_cov(modes, cl4)
    F = S @ np.linalg.inv(S + lam * tau * omega * np.eye(len(modes)))
    return F @ (omega * (Y.T @ Ib @ Y))
