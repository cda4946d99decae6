"""Host checks of the seeded input generator (no GPU)."""
import numpy as np

from oracle import healpix
from paper_1211_0585_amd import synth


def test_disc_mask_band_search_equals_full_scan():
    """The disc mask restricted to each disc's colatitude band equals a scan of
    every pixel (the generator falls back to the scan for unsorted input)."""
    th, ph = healpix.pixel_angles(64)
    fast = synth.disc_holes(th, ph, 300, 1.5, 4)
    rev = np.arange(th.size)[::-1]
    full = synth.disc_holes(th[rev], ph[rev], 300, 1.5, 4)[rev]
    assert np.array_equal(fast, full) and fast.any()


def test_streams_are_reproducible_and_distinct():
    a = synth.rng(3, 0).standard_normal(8)
    assert np.array_equal(a, synth.rng(3, 0).standard_normal(8))
    assert not np.allclose(a, synth.rng(3, 1).standard_normal(8))
