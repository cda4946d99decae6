"""FP64 CPU oracle for the messenger-field Wiener filter (test infrastructure).

This package is a plain, slow, obviously correct reference implementation of
what the GPU path computes. It exists only to check that path: the tests, the
smoke check and the CPU-baseline leg of the benchmark may import it; the
product library never does, and it shares no code with the HIP kernels.

Modules
  healpix   ring geometry of the HEALPix RING scheme
  legendre  normalised associated Legendre functions by the l-recurrence
  sht       ring DFTs and the spherical-harmonic transform pair
  messenger the messenger iteration of Elsner & Wandelt, Sect. 2, Eqs. (3)-(4)
  dense     dense linear-algebra solves at tiny Nside (Eq. 2 and the fixed point)

Every function names the passage of the paper (or the public definition) it
follows. Functions without an independent pin say "parity unpinned".
"""
