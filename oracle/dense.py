"""Dense linear-algebra solves at tiny Nside (oracle; test infrastructure only).

Everything here works in the real orthonormal harmonic basis
  x_l0,  x_lm^c,  x_lm^s  (m > 0)   with basis functions
  lambda_l0(z),  sqrt(2) lambda_lm(z) cos(m phi),  sqrt(2) lambda_lm(z) sin(m phi)
so that the complex coefficients of a real field are a_l0 = x_l0 and
a_lm = (x_lm^c - i x_lm^s) / sqrt(2). Y is the synthesis matrix (pixels x modes),
C = diag(C_l) the signal covariance (modes with C_l = 0 are left out: the signal
has no such component) and N^-1 = diag(ninv) the pixel noise precision.

  wiener_dense          Eq. (2): (S^-1 + N^-1) s = N^-1 d, written in the harmonic
                        basis as [C^-1 + Y^T N^-1 Y] x = Y^T N^-1 d, s = Y x.
  messenger_fixed_point the exact fixed point of one sweep of Eqs. (3)-(4) at a
                        fixed lambda, with the analysis Omega Y^T:
                        [C^-1 + Y^T N_l^-1 Y + (lambda tau Omega)^-1 (I - Omega Y^T Y)] x
                            = Y^T N_l^-1 d,
                        N_l^-1 = ninv / (1 + (lambda - 1) tau ninv).
                        It equals Eq. (2) when Omega Y^T Y = I and lambda = 1.
  iteration_matrix      M with x_{k+1} = M x_k + const for one sweep; the paper
                        states the iteration converges unconditionally
                        (Sect. 2), i.e. spectral radius < 1.
"""
import numpy as np

from . import healpix
from .legendre import lambda_all, alm_index, n_alm
from .messenger import tau_of, pixel_weight, harmonic_filter


def real_modes(lmax, cl=None):
    """List of (l, m, kind) for the real basis; kind 0 = m=0, 1 = cos, 2 = sin.
    Modes with cl[l] <= 0 are dropped when cl is given."""
    out = []
    for l in range(lmax + 1):
        if cl is not None and not cl[l] > 0:
            continue
        out.append((l, 0, 0))
        for m in range(1, l + 1):
            out.append((l, m, 1))
            out.append((l, m, 2))
    return out


def synthesis_matrix(nside, lmax, modes):
    """Y[p, k]: value of real basis function k at pixel p."""
    theta, phi = healpix.pixel_angles(nside)
    z = np.cos(theta)
    lam = lambda_all(lmax, z)                       # [N_lm, npix]
    Y = np.empty((z.size, len(modes)))
    for k, (l, m, kind) in enumerate(modes):
        row = lam[alm_index(lmax, l, m)]
        if kind == 0:
            Y[:, k] = row
        elif kind == 1:
            Y[:, k] = np.sqrt(2.0) * row * np.cos(m * phi)
        else:
            Y[:, k] = np.sqrt(2.0) * row * np.sin(m * phi)
    return Y


def x_to_alm(x, modes, lmax):
    """Real-basis coefficients -> packed complex alm (missing modes are zero)."""
    alm = np.zeros(n_alm(lmax), dtype=np.complex128)
    for k, (l, m, kind) in enumerate(modes):
        i = alm_index(lmax, l, m)
        if kind == 0:
            alm[i] += x[k]
        elif kind == 1:
            alm[i] += x[k] / np.sqrt(2.0)
        else:
            alm[i] += -1j * x[k] / np.sqrt(2.0)
    return alm


def _cdiag(modes, cl):
    return np.array([cl[l] for (l, _, _) in modes], dtype=np.float64)


def wiener_dense(d, ninv, cl, nside, lmax):
    """Textbook Wiener filter, Eq. (2), by a dense solve. Returns (map, alm)."""
    modes = real_modes(lmax, cl)
    Y = synthesis_matrix(nside, lmax, modes)
    ninv = np.asarray(ninv, dtype=np.float64)
    A = np.diag(1.0 / _cdiag(modes, cl)) + Y.T @ (ninv[:, None] * Y)
    x = np.linalg.solve(A, Y.T @ (ninv * d))
    return Y @ x, x_to_alm(x, modes, lmax)


def messenger_fixed_point(d, ninv, cl, lam, nside, lmax):
    """Fixed point of the messenger sweep at a fixed lambda. Returns (map, alm)."""
    modes = real_modes(lmax, cl)
    Y = synthesis_matrix(nside, lmax, modes)
    ninv = np.asarray(ninv, dtype=np.float64)
    tau = tau_of(ninv)
    omega = healpix.pixel_area(nside)
    nl = ninv / (1.0 + (lam - 1.0) * tau * ninv)
    n = len(modes)
    A = (np.diag(1.0 / _cdiag(modes, cl)) + Y.T @ (nl[:, None] * Y)
         + (np.eye(n) - omega * (Y.T @ Y)) / (lam * tau * omega))
    x = np.linalg.solve(A, Y.T @ (nl * d))
    return Y @ x, x_to_alm(x, modes, lmax)


def iteration_matrix(ninv, cl, lam, nside, lmax):
    """M = F Omega Y^T (I - W) Y: one sweep maps x_k to M x_k + const."""
    modes = real_modes(lmax, cl)
    Y = synthesis_matrix(nside, lmax, modes)
    ninv = np.asarray(ninv, dtype=np.float64)
    tau = tau_of(ninv)
    omega = healpix.pixel_area(nside)
    w = pixel_weight(ninv, lam, tau)
    f = harmonic_filter(np.asarray(cl, dtype=np.float64), lam, tau, omega)
    fd = np.array([f[l] for (l, _, _) in modes])
    return fd[:, None] * (omega * (Y.T @ ((1.0 - w)[:, None] * Y)))


def gram_matrix(nside, lmax):
    """(Omega Y^T Y, modes): the Gram matrix of the real basis functions l <= lmax under
    the pixel-area sum (the identity for an exact quadrature)."""
    modes = real_modes(lmax)
    Y = synthesis_matrix(nside, lmax, modes)
    return healpix.pixel_area(nside) * (Y.T @ Y), modes


def gram_defect(nside, lmax):
    """|| I - Omega Y^T Y ||_2 over all modes l <= lmax: how far the pixel-area
    analysis is from inverting the synthesis (zero for an exact quadrature)."""
    G, modes = gram_matrix(nside, lmax)
    return float(np.linalg.norm(np.eye(len(modes)) - G, 2))
