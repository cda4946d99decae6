"""Write the stored expected values of the Nside-1024 / lmax-2048 precision tests.

Calls only the FP64 oracle and the seeded input generator: the satellite-scale
recipe at Nside 1024 with N_obs scaled by 1/4 (seed 0, model seed 0), d = oracle
synthesis of the drawn signal + noise, then the oracle messenger solve under a
short schedule that ends at lambda = 1 (a full 80-sweep oracle solve at this size
would take many hours). Stores, for d and for the result after the schedule:
the norm, first entries and seeded random projections, seeded samples of pixels
and alm, and the L2 norm and a seeded random projection of every ring of the map and of
every m column of the alm (so that an error confined to a few rings or a few m cannot hide under the
global norm).

Run from the repository root:  python tests/golden/make_golden_1024.py
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import healpix, messenger, sht  # noqa: E402
from oracle.legendre import alm_index  # noqa: E402
from paper_1211_0585_amd import synth  # noqa: E402

NSIDE, LMAX = 1024, 2048
SCHEDULE = np.array([100.0, 10.0, 1.0, 1.0])
OUT = os.path.join(ROOT, "tests", "golden", "nside1024_satellite.npz")


def ring_norms(s_map, nside):
    g = healpix.ring_info(nside)
    return np.array([np.linalg.norm(s_map[s:s + n]) for s, n in zip(g["start"], g["nphi"])])


def m_norms(s_alm, lmax):
    """sqrt(sum_l w_m |a_lm|^2) for every m (w = 1 at m = 0, else 2)."""
    out = np.empty(lmax + 1)
    for m in range(lmax + 1):
        i0 = alm_index(lmax, m, m)
        col = s_alm[i0:i0 + lmax - m + 1]
        out[m] = np.sqrt((1.0 if m == 0 else 2.0) * np.sum(np.abs(col) ** 2))
    return out


def summarize(prefix, s_map, s_alm, store):
    rs = np.random.default_rng(2024)
    pix = np.sort(rs.choice(s_map.size, 8192, replace=False))
    alm_idx = np.sort(rs.choice(s_alm.size, 8192, replace=False))
    w = sht.alm_weights(LMAX)
    store[prefix + "pix_idx"] = pix
    store[prefix + "pix_val"] = s_map[pix]
    store[prefix + "alm_idx"] = alm_idx
    store[prefix + "alm_val"] = s_alm[alm_idx]
    store[prefix + "map_norm"] = np.linalg.norm(s_map)
    store[prefix + "alm_norm"] = np.sqrt(np.sum(w * np.abs(s_alm) ** 2))
    store[prefix + "ring_norm"] = ring_norms(s_map, NSIDE)
    store[prefix + "m_norm"] = m_norms(s_alm, LMAX)
    # per ring and per m: the projection on one seeded random vector (a local error
    # changes it by about its own size, whatever the sign)
    v = np.random.default_rng(99).standard_normal(s_map.size)
    g = healpix.ring_info(NSIDE)
    store[prefix + "ring_proj"] = np.array([np.dot(v[a:a + n], s_map[a:a + n]) for a, n in zip(g["start"], g["nphi"])])
    u = np.random.default_rng(98).standard_normal(s_alm.size) + 1j * np.random.default_rng(97).standard_normal(s_alm.size)
    mp = np.empty(LMAX + 1, dtype=np.complex128)
    for m in range(LMAX + 1):
        i0 = alm_index(LMAX, m, m)
        mp[m] = np.sum(u[i0:i0 + LMAX - m + 1] * s_alm[i0:i0 + LMAX - m + 1])
    store[prefix + "m_proj"] = mp
    proj = np.random.default_rng(77).standard_normal((4, s_map.size))
    store[prefix + "map_proj"] = proj @ s_map


def main():
    t0 = time.time()
    theta, phi = healpix.pixel_angles(NSIDE)
    c = synth.satellite_case(theta, phi, LMAX, seed=0, nobs_scale=0.25)
    d = sht.alm2map(c["signal_alm"], NSIDE, LMAX) + c["noise"]
    store = {"d_norm": np.linalg.norm(d), "d_head": d[:64].copy(),
             "d_proj": np.random.default_rng(77).standard_normal((4, d.size)) @ d,
             "schedule": SCHEDULE}
    print(f"inputs ready ({time.time() - t0:.0f} s)", flush=True)

    def cb(k, s, a):
        print(f"sweep {k + 1}/{len(SCHEDULE)} ({time.time() - t0:.0f} s)", flush=True)

    sf, af = messenger.solve(d, c["ninv"], c["cl"], SCHEDULE, NSIDE, LMAX, callback=cb)
    summarize("sol_", sf, af, store)
    np.savez_compressed(OUT, **store)
    print(f"wrote {OUT} ({time.time() - t0:.0f} s)", flush=True)


if __name__ == "__main__":
    main()
