"""GPU parity of constrained realisations (wf_constrained_batch; Sect. 3: Wiener filter
plus fluctuation map) against the oracle.

  * s_CR and its alm vs oracle.constrained.constrained_messenger on the same data,
    unit draws and lambda schedule: FP64 within 1e-10, FP32 and bf16x6 within 1e-5;
    three maps with their own draws in one batch, each equal to its solo run.
  * Nside 512 (FP64, the full-size plan): s_CR(d) - WF(d) equals s_CR(0) for the
    same draws (the filter is linear), and draws of zero give WF(d) bit for bit.
"""
import sys

import numpy as np
import pytest

from oracle import constrained, healpix
from paper_1211_0585_amd import synth
from tests.helpers import alm_rel_l2, rel_l2, small_band_inputs

pytestmark = pytest.mark.gpu


def _log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_1211_0585_amd import mwf
    mwf.lib()
    return torch


TOL = {0: 1e-10, 1: 1e-5, 3: 1e-5}


@pytest.mark.parametrize("name,dt", [("f64", 0), ("f32", 1), ("bf16x6", 3)])
@pytest.mark.parametrize("nside,lmax", [(16, 32), (32, 64)])
def test_constrained_parity(torch_dev, name, dt, nside, lmax):
    torch = torch_dev
    from paper_1211_0585_amd import mwf
    nm = 3
    cs = [small_band_inputs(nside, lmax, seed=60 + i) for i in range(nm)]
    c = cs[0]
    npix = healpix.npix(nside)
    xi, eta = synth.fluctuation_draws(npix, lmax, 21, nmaps=nm)
    lams = np.geomspace(1e3, 1.0, 24)
    rt = np.float64 if dt == 0 else np.float32
    ct = np.complex128 if dt == 0 else np.complex64
    D = np.stack([x["d"] for x in cs]).astype(rt)
    X, E = xi.astype(ct), eta.astype(rt)
    with mwf.Plan(nside, lmax, c["cl"], c["ninv"], dtype=dt, max_batch=nm) as p:
        dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
        s, a = p.constrained(dev(D), dev(X), dev(E), lams)
        s1, a1 = p.constrained(dev(D[1]), dev(X[1]), dev(E[1]), lams)
        p.sync()
        s, a, s1, a1 = (t.cpu().numpy() for t in (s, a, s1, a1))
    for i in range(nm):
        m_ref, a_ref = constrained.constrained_messenger(D[i].astype(np.float64), c["ninv"], c["cl"],
                                                         X[i].astype(np.complex128), E[i].astype(np.float64),
                                                         lams, nside, lmax)
        e_m, e_a = rel_l2(s[i], m_ref), alm_rel_l2(a[i], a_ref, lmax)
        _log(f"constrained {name} Nside {nside} map {i}: map {e_m:.2e} alm {e_a:.2e}")
        assert e_m <= TOL[dt] and e_a <= TOL[dt]
    assert rel_l2(s1, s[1]) <= 1e-12 and alm_rel_l2(a1, a[1], lmax) <= 1e-12


def test_constrained_nside512_linearity(torch_dev):
    torch = torch_dev
    from paper_1211_0585_amd import mwf
    nside, lmax = 512, 1024
    theta, phi = healpix.pixel_angles(nside)
    c = synth.satellite_case(theta, phi, lmax, seed=0)
    xi, eta = synth.fluctuation_draws(c["ninv"].size, lmax, 31)
    lams = np.geomspace(1e4, 1.0, 12)
    with mwf.Plan(nside, lmax, c["cl"], c["ninv"]) as p:
        d = p.alm2map(torch.from_numpy(c["signal_alm"]).cuda()) + torch.from_numpy(c["noise"]).cuda()
        X, E = torch.from_numpy(xi[0]).cuda(), torch.from_numpy(eta[0]).cuda()
        s_cr, a_cr = p.constrained(d, X, E, lams)
        s_0, a_0 = p.constrained(torch.zeros_like(d), X, E, lams)
        s_wf, a_wf = p.solve(d, lams)
        z_cr, z_a = p.constrained(d, torch.zeros_like(X), torch.zeros_like(E), lams)
        p.sync()
        s_cr, a_cr, s_0, a_0, s_wf, a_wf, z_cr, z_a = (t.cpu().numpy() for t in
                                                        (s_cr, a_cr, s_0, a_0, s_wf, a_wf, z_cr, z_a))
    e_m = rel_l2(s_cr - s_wf, s_0)
    e_a = alm_rel_l2(a_cr - a_wf, a_0, lmax)
    _log(f"constrained Nside 512: CR(d) - WF(d) vs CR(0): map {e_m:.2e} alm {e_a:.2e}; "
         f"|fluctuation| / |WF| = {np.linalg.norm(s_0) / np.linalg.norm(s_wf):.3f}")
    assert e_m <= 1e-10 and e_a <= 1e-10
    assert np.array_equal(z_cr, s_wf) and np.array_equal(z_a, a_wf)
