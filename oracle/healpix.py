"""HEALPix RING-scheme geometry (oracle; test infrastructure only).

The paper leaves the pixelisation open (Sect. 2 changes basis "e.g. to Fourier
space"); on the sphere the map lives on HEALPix pixels in RING order, whose
geometry is the public definition of Gorski et al. 2005 (ApJ 622, 759),
Sect. 4 / Eqs. (4)-(10) there:

  rings i = 1 .. 4 Nside - 1, counted from the north pole
  north cap (i < Nside):      n_phi = 4 i,     z = 1 - i^2 / (3 Nside^2),
                              phi_j = pi (j + 1/2) / (2 i)
  belt (Nside <= i <= 3Nside): n_phi = 4 Nside, z = 4/3 - 2 i / (3 Nside),
                              phi_j = pi (j + s_i / 2) / (2 Nside),
                              s_i = (i - Nside + 1) mod 2
  south cap (i > 3 Nside):    mirror of ring 4 Nside - i, z -> -z
"""
import numpy as np


def npix(nside):
    return 12 * nside * nside


def pixel_area(nside):
    """Solid angle of one pixel, 4 pi / npix (all HEALPix pixels are equal-area)."""
    return 4.0 * np.pi / npix(nside)


def ring_info(nside):
    """Per-ring arrays for rings i = 1..4*nside-1 (index r = i-1).

    Returns a dict with
      z     cos(theta) of the ring (float64)
      nphi  number of pixels in the ring (int64)
      phi0  longitude of the ring's first pixel (float64)
      start index of the ring's first pixel in RING order (int64)
    """
    n = int(nside)
    nr = 4 * n - 1
    z = np.empty(nr)
    nphi = np.empty(nr, dtype=np.int64)
    phi0 = np.empty(nr)
    start = np.empty(nr, dtype=np.int64)
    total = 12 * n * n
    for r in range(nr):
        i = r + 1
        if i < n:                       # north polar cap
            z[r] = 1.0 - i * i / (3.0 * n * n)
            nphi[r] = 4 * i
            phi0[r] = np.pi / (4.0 * i)
            start[r] = 2 * i * (i - 1)
        elif i <= 3 * n:                # equatorial belt
            z[r] = 2.0 * (2 * n - i) / (3.0 * n)     # = 4/3 - 2 i / (3 Nside)
            nphi[r] = 4 * n
            s = (i - n + 1) % 2
            phi0[r] = np.pi * s / (4.0 * n)
            start[r] = 2 * n * (n - 1) + 4 * n * (i - n)
        else:                           # south polar cap, mirror of ring 4n - i
            ip = 4 * n - i
            z[r] = -(1.0 - ip * ip / (3.0 * n * n))
            nphi[r] = 4 * ip
            phi0[r] = np.pi / (4.0 * ip)
            start[r] = total - 2 * ip * (ip + 1)
    return {"z": z, "nphi": nphi, "phi0": phi0, "start": start}


def pixel_angles(nside):
    """(theta, phi) of every pixel centre in RING order."""
    g = ring_info(nside)
    theta = np.empty(npix(nside))
    phi = np.empty(npix(nside))
    for r in range(len(g["z"])):
        s, n = g["start"][r], g["nphi"][r]
        theta[s:s + n] = np.arccos(g["z"][r])
        phi[s:s + n] = g["phi0"][r] + 2.0 * np.pi * np.arange(n) / n
    return theta, phi
