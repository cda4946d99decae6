"""Write the stored expected values of the full-size polarised tests.

Calls only the FP64 polarised oracle and the seeded input generator: the
satellite-scale polarised case at Nside 512 / lmax 1024 (seed 0, model seed 0:
the temperature recipe of the satellite case, cl_pol spectra, P noise twice the T
variance with Q-U correlations, T mask |b| < 15 deg plus discs, P mask |b| < 20 deg
plus the same discs), d = oracle synthesis of the drawn T/E/B alm + noise, then the
oracle's polarised messenger solve under a short schedule ending at lambda = 1.
Stores, for d and for the result: norms, first entries and seeded projections of
each field, seeded samples of pixels and alm, and per field the norm and a seeded
projection of every ring and of every m column.

Run from the repository root:  python tests/golden/make_golden_pol.py
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import healpix, polar, sht  # noqa: E402
from oracle.legendre import alm_index  # noqa: E402
from paper_1211_0585_amd import synth  # noqa: E402

NSIDE, LMAX = 512, 1024
SCHEDULE = np.array([100.0, 10.0, 1.0])
OUT = os.path.join(ROOT, "tests", "golden", "nside512_pol.npz")


def summarize(prefix, maps, alm, store):
    g = healpix.ring_info(NSIDE)
    rs = np.random.default_rng(2024)
    pix = np.sort(rs.choice(maps.shape[1], 4096, replace=False))
    aidx = np.sort(rs.choice(alm.shape[1], 4096, replace=False))
    w = sht.alm_weights(LMAX)
    v = np.random.default_rng(99).standard_normal(maps.shape[1])
    u = np.random.default_rng(98).standard_normal(alm.shape[1]) + 1j * np.random.default_rng(97).standard_normal(
        alm.shape[1])
    proj = np.random.default_rng(77).standard_normal((2, maps.shape[1]))
    store[prefix + "pix_idx"] = pix
    store[prefix + "alm_idx"] = aidx
    for f in range(3):
        key = prefix + "TQU"[f] + "_"
        keya = prefix + "TEB"[f] + "_"
        store[key + "pix_val"] = maps[f, pix]
        store[key + "map_norm"] = np.linalg.norm(maps[f])
        store[key + "map_proj"] = proj @ maps[f]
        store[key + "ring_norm"] = np.array([np.linalg.norm(maps[f, a:a + n]) for a, n in zip(g["start"], g["nphi"])])
        store[key + "ring_proj"] = np.array([np.dot(v[a:a + n], maps[f, a:a + n]) for a, n in zip(g["start"], g["nphi"])])
        store[keya + "alm_val"] = alm[f, aidx]
        store[keya + "alm_norm"] = np.sqrt(np.sum(w * np.abs(alm[f]) ** 2))
        mn = np.empty(LMAX + 1)
        mp = np.empty(LMAX + 1, dtype=np.complex128)
        for m in range(LMAX + 1):
            i0 = alm_index(LMAX, m, m)
            col = alm[f, i0:i0 + LMAX - m + 1]
            mn[m] = np.sqrt((1.0 if m == 0 else 2.0) * np.sum(np.abs(col) ** 2))
            mp[m] = np.sum(u[i0:i0 + LMAX - m + 1] * col)
        store[keya + "m_norm"] = mn
        store[keya + "m_proj"] = mp


def main():
    t0 = time.time()
    theta, phi = healpix.pixel_angles(NSIDE)
    c = synth.pol_satellite_case(theta, phi, LMAX, seed=0)
    d = polar.alm2map(c["signal_alm"], NSIDE, LMAX) + c["noise"]
    store = {"schedule": SCHEDULE}
    summarize("d_", d, polar.map2alm(d, NSIDE, LMAX), store)
    print(f"inputs ready ({time.time() - t0:.0f} s)", flush=True)

    def cb(k, s, a):
        print(f"sweep {k + 1}/{len(SCHEDULE)} ({time.time() - t0:.0f} s)", flush=True)

    s_map, s_alm = polar.solve(d, c["ninv6"], c["cl4"], SCHEDULE, NSIDE, LMAX, mask=c["mask"], callback=cb)
    summarize("sol_", s_map, s_alm, store)
    np.savez_compressed(OUT, **store)
    print(f"wrote {OUT} ({time.time() - t0:.0f} s)", flush=True)


if __name__ == "__main__":
    main()
