"""Write the stored expected values of the full-size (Nside 512, lmax 1024) tests.

Calls only the FP64 oracle and the seeded input generator: the satellite-scale
case (seed 0, model seed 0), d = oracle synthesis of the drawn signal + noise,
then the oracle messenger solve for the first 2 sweeps and for the full
80-sweep schedule. Stores the norm, first entries and seeded random projections
of d (so a test can check an input it builds itself), sampled outputs (seeded
pixel and alm indices), the norms of the full outputs and their projections on
seeded random vectors, and per ring and per m the norm and the projection on one
seeded random vector.

Run from the repository root:  python tests/golden/make_golden.py
(about an hour on 8 CPU cores).
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
from make_golden_1024 import m_norms, ring_norms  # noqa: E402  (same directory)

NSIDE, LMAX = 512, 1024
OUT = os.path.join(ROOT, "tests", "golden", "nside512_satellite.npz")


def summarize(prefix, s_map, s_alm, store):
    rs = np.random.default_rng(2024)
    pix = np.sort(rs.choice(s_map.size, 4096, replace=False))
    alm_idx = np.sort(rs.choice(s_alm.size, 4096, replace=False))
    w = sht.alm_weights(LMAX)
    store[prefix + "pix_idx"] = pix
    store[prefix + "pix_val"] = s_map[pix]
    store[prefix + "alm_idx"] = alm_idx
    store[prefix + "alm_val"] = s_alm[alm_idx]
    store[prefix + "map_norm"] = np.linalg.norm(s_map)
    store[prefix + "alm_norm"] = np.sqrt(np.sum(w * np.abs(s_alm) ** 2))
    proj = np.random.default_rng(77).standard_normal((4, s_map.size))
    store[prefix + "map_proj"] = proj @ s_map
    # per ring and per m: norms, and the projection on one seeded random vector (a local
    # error changes it by about its own size, whatever the sign)
    store[prefix + "ring_norm"] = ring_norms(s_map, NSIDE)
    store[prefix + "m_norm"] = m_norms(s_alm, LMAX)
    v = np.random.default_rng(99).standard_normal(s_map.size)
    g = healpix.ring_info(NSIDE)
    store[prefix + "ring_proj"] = np.array([np.dot(v[a:a + n], s_map[a:a + n]) for a, n in zip(g["start"], g["nphi"])])
    u = np.random.default_rng(98).standard_normal(s_alm.size) + 1j * np.random.default_rng(97).standard_normal(s_alm.size)
    mp = np.empty(LMAX + 1, dtype=np.complex128)
    for m in range(LMAX + 1):
        i0 = alm_index(LMAX, m, m)
        mp[m] = np.sum(u[i0:i0 + LMAX - m + 1] * s_alm[i0:i0 + LMAX - m + 1])
    store[prefix + "m_proj"] = mp


def main():
    t0 = time.time()
    theta, phi = healpix.pixel_angles(NSIDE)
    c = synth.satellite_case(theta, phi, LMAX, seed=0)
    d = sht.alm2map(c["signal_alm"], NSIDE, LMAX) + c["noise"]
    store = {"d_norm": np.linalg.norm(d), "d_head": d[:64].copy(),
             "d_proj": np.random.default_rng(77).standard_normal((4, d.size)) @ d}
    print(f"inputs ready ({time.time() - t0:.0f} s)", flush=True)
    sched = c["schedule"]
    s2, a2 = messenger.solve(d, c["ninv"], c["cl"], sched[:2], NSIDE, LMAX)
    summarize("two_", s2, a2, store)
    print(f"2 sweeps done ({time.time() - t0:.0f} s)", flush=True)

    def cb(k, s, a):
        print(f"sweep {k + 1}/{len(sched)} ({time.time() - t0:.0f} s)", flush=True)

    sf, af = messenger.solve(d, c["ninv"], c["cl"], sched, NSIDE, LMAX, callback=cb)
    summarize("full_", sf, af, store)
    np.savez_compressed(OUT, **store)
    print(f"wrote {OUT} ({time.time() - t0:.0f} s)", flush=True)


if __name__ == "__main__":
    main()
