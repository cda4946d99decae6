"""GPU edge and degenerate cases of the FP64 path against the oracle and against
exact properties of the method:

* band limits at both ends: lmax = 0 (monopole only) and lmax = 4 nside - 1, the
  largest the ring layout accepts (every ring aliases);
* C_l = 0 for every l: the filter removes everything and s_WF is exactly zero;
* one observed pixel (all others masked), one sweep, a huge lambda (the filter and
  the pixel weight both tend to zero);
* a mask given as an argument equals the same pixels given N^-1 = 0 (bitwise);
* linearity in d for a fixed schedule (Eq. 3 and 4 are linear in d);
* a batch of 2 maps on a plan sized for 5 equals the maps solved one by one.
"""
import sys

import numpy as np
import pytest

from oracle import healpix, messenger, sht
from tests.helpers import alm_rel_l2, random_alm, rel_l2, small_band_inputs

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


@pytest.mark.parametrize("nside,lmax", [(1, 0), (2, 0), (1, 3), (2, 7), (4, 15), (8, 31)])
def test_sht_band_limit_extremes(torch_dev, nside, lmax):
    torch = torch_dev
    from paper_1211_0585_amd import mwf
    npix = 12 * nside * nside
    f = np.random.default_rng(nside + lmax).standard_normal(npix)
    a = random_alm(lmax, 3 * nside + lmax)
    with mwf.Plan(nside, lmax, np.ones(lmax + 1), np.ones(npix)) as p:
        g_alm = p.map2alm(torch.from_numpy(f).cuda()).cpu().numpy()
        g_map = p.alm2map(torch.from_numpy(a).cuda()).cpu().numpy()
        p.sync()
    e1 = alm_rel_l2(g_alm, sht.map2alm(f, nside, lmax), lmax)
    e2 = rel_l2(g_map, sht.alm2map(a, nside, lmax))
    _log(f"Nside {nside} lmax {lmax}: map2alm {e1:.2e}, alm2map {e2:.2e}")
    assert e1 <= 1e-12 and e2 <= 1e-12


def test_zero_spectrum_gives_zero(torch_dev):
    torch = torch_dev
    from paper_1211_0585_amd import mwf
    c = small_band_inputs(16, 32, seed=3)
    with mwf.Plan(16, 32, np.zeros(33), c["ninv"]) as p:
        s, a = p.solve(torch.from_numpy(c["d"]).cuda(), c["schedule"][:10])
        p.sync()
        assert not torch.any(s != 0) and not torch.any(a != 0)


@pytest.mark.parametrize("case", ["one_pixel", "one_sweep", "huge_lambda"])
def test_degenerate_solves_vs_oracle(torch_dev, case):
    torch = torch_dev
    from paper_1211_0585_amd import mwf
    nside, lmax = 8, 16
    c = small_band_inputs(nside, lmax, seed=9)
    ninv, lams = c["ninv"].copy(), np.geomspace(1e3, 1.0, 6)
    if case == "one_pixel":
        keep = int(np.argmax(ninv))
        ninv = np.zeros_like(ninv)
        ninv[keep] = 2.0
    elif case == "one_sweep":
        lams = np.array([3.0])
    else:
        lams = np.full(3, 1e12)
    with mwf.Plan(nside, lmax, c["cl"], ninv) as p:
        s, a = p.solve(torch.from_numpy(c["d"]).cuda(), lams)
        p.sync()
        s, a = s.cpu().numpy(), a.cpu().numpy()
    ref_s, ref_a = messenger.solve(c["d"], ninv, c["cl"], lams, nside, lmax)
    e = max(rel_l2(s, ref_s), alm_rel_l2(a, ref_a, lmax))
    _log(f"{case}: rel diff {e:.2e}, |s| {np.linalg.norm(ref_s):.3e}")
    assert e <= 1e-10


def test_mask_argument_equals_zero_inverse_noise(torch_dev):
    torch = torch_dev
    from paper_1211_0585_amd import mwf
    nside, lmax = 16, 32
    c = small_band_inputs(nside, lmax, seed=4)
    theta, _ = healpix.pixel_angles(nside)
    mask = np.abs(theta - 1.2) > 0.3            # 1 = observed
    ninv_full = np.where(c["ninv"] > 0, c["ninv"], 1.0)
    d = torch.from_numpy(c["d"]).cuda()
    lams = np.geomspace(1e3, 1.0, 8)
    with mwf.Plan(nside, lmax, c["cl"], ninv_full, mask=mask) as p:
        s1, _ = p.solve(d, lams)
        p.sync()
        s1 = s1.cpu().numpy()
    with mwf.Plan(nside, lmax, c["cl"], np.where(mask, ninv_full, 0.0)) as p:
        s2, _ = p.solve(d, lams)
        p.sync()
        s2 = s2.cpu().numpy()
    assert np.array_equal(s1, s2)


def test_linearity_in_data(torch_dev):
    torch = torch_dev
    from paper_1211_0585_amd import mwf
    nside, lmax = 32, 64
    c1 = small_band_inputs(nside, lmax, seed=11)
    c2 = small_band_inputs(nside, lmax, seed=12)
    al, be = 0.75, -2.5
    lams = np.geomspace(1e3, 1.0, 10)
    with mwf.Plan(nside, lmax, c1["cl"], c1["ninv"]) as p:
        out = []
        for d in (c1["d"], c2["d"], al * c1["d"] + be * c2["d"]):
            s, _ = p.solve(torch.from_numpy(d).cuda(), lams)
            p.sync()
            out.append(s.cpu().numpy())
    e = rel_l2(out[2], al * out[0] + be * out[1])
    _log(f"linearity: {e:.2e}")
    assert e <= 1e-12


def test_partial_batch_equals_single(torch_dev):
    torch = torch_dev
    from paper_1211_0585_amd import mwf
    nside, lmax = 16, 32
    cs = [small_band_inputs(nside, lmax, seed=20 + i) for i in range(2)]
    d = np.stack([c["d"] for c in cs])
    lams = np.geomspace(1e2, 1.0, 5)
    with mwf.Plan(nside, lmax, cs[0]["cl"], cs[0]["ninv"], max_batch=5) as p:
        sb, _ = p.solve(torch.from_numpy(d).cuda(), lams)
        p.sync()
        for i in range(2):
            s1, _ = p.solve(torch.from_numpy(d[i].copy()).cuda(), lams)
            p.sync()
            assert torch.equal(s1, sb[i])
        with pytest.raises(mwf.WFError):
            p.solve(torch.zeros((6, 12 * nside * nside), dtype=torch.float64, device="cuda"), lams)
