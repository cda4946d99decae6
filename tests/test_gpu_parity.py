"""GPU parity of the FP64 path against the oracle (element by element).

Every call goes through the C ABI (libmwf.so via the ctypes binding); inputs
are identical seeded arrays on both sides. Bars: FP64 SHTs <= 1e-12 relative L2,
FP64 wf_solve <= 1e-10 relative L2 on s_WF and the alm.
"""
import sys

import numpy as np
import pytest

from oracle import healpix, messenger, sht
from tests.helpers import alm_rel_l2, random_alm, rel_l2, small_band_inputs

pytestmark = pytest.mark.gpu

SHT_TOL = 1e-12
SOLVE_TOL = 1e-10


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_1211_0585_amd import mwf
    mwf.lib()
    return torch


def _plan(nside, lmax, cl=None, ninv=None, mask=None, max_batch=1):
    from paper_1211_0585_amd import mwf
    if cl is None:
        cl = np.ones(lmax + 1)
    if ninv is None:
        ninv = np.ones(12 * nside * nside)
    return mwf.Plan(nside, lmax, cl, ninv, mask=mask, max_batch=max_batch)


def _log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("nside,lmax", [(1, 2), (2, 7), (4, 8), (4, 15), (8, 16), (16, 32),
                                        (16, 47), (32, 64), (64, 128), (128, 256), (256, 300)])
def test_sht_pair_parity(torch_dev, nside, lmax):
    torch = torch_dev
    _log("sht parity", nside, lmax)
    rs = np.random.default_rng(nside * 7 + lmax)
    f = rs.standard_normal(12 * nside * nside)
    a = random_alm(lmax, nside + lmax)
    with _plan(nside, lmax) as p:
        g_alm = p.map2alm(torch.from_numpy(f).cuda())
        g_map = p.alm2map(torch.from_numpy(a).cuda())
        torch.cuda.synchronize()
        p.sync()
        ref_alm = sht.map2alm(f, nside, lmax)
        ref_map = sht.alm2map(a, nside, lmax)
        e1 = alm_rel_l2(g_alm.cpu().numpy(), ref_alm, lmax)
        e2 = rel_l2(g_map.cpu().numpy(), ref_map)
        _log("  map2alm err", e1, "alm2map err", e2)
        assert e1 <= SHT_TOL
        assert e2 <= SHT_TOL


@pytest.mark.parametrize("nside,lmax,nmaps", [(32, 48, 5), (256, 64, 4)])
def test_sht_pair_parity_batched_ring_classes(torch_dev, nside, lmax, nmaps):
    """From 4 maps on the ring transforms run in the batched launch classes (one wave per
    ring pair up to 1024 points, the other classes beyond): every map of such a batch
    against the oracle, both directions. At Nside 256 the mixed-radix rings of more than 512
    points (e.g. 540 = 4 * 135) run in the class of the long rings, the shorter ones and the
    Bluestein rings of up to 1024 points one wave per pair."""
    torch = torch_dev
    _log("sht batched classes", nside, lmax, nmaps)
    rs = np.random.default_rng(nside + 11 * nmaps)
    f = rs.standard_normal((nmaps, 12 * nside * nside))
    a = np.stack([random_alm(lmax, 100 * nside + k) for k in range(nmaps)])
    with _plan(nside, lmax, max_batch=nmaps) as p:
        g_alm = p.map2alm(torch.from_numpy(f).cuda()).cpu().numpy()
        g_map = p.alm2map(torch.from_numpy(a).cuda()).cpu().numpy()
        p.sync()
    for k in range(nmaps):
        e1 = alm_rel_l2(g_alm[k], sht.map2alm(f[k], nside, lmax), lmax)
        e2 = rel_l2(g_map[k], sht.alm2map(a[k], nside, lmax))
        _log("  map", k, "map2alm err", e1, "alm2map err", e2)
        assert e1 <= SHT_TOL
        assert e2 <= SHT_TOL


def test_sht_batch_matches_single(torch_dev):
    torch = torch_dev
    nside, lmax = 32, 64
    rs = np.random.default_rng(5)
    f = rs.standard_normal((3, 12 * nside * nside))
    with _plan(nside, lmax, max_batch=3) as p:
        batch = p.map2alm(torch.from_numpy(f).cuda()).cpu().numpy()
        for i in range(3):
            one = p.map2alm(torch.from_numpy(f[i].copy()).cuda()).cpu().numpy()
            assert np.array_equal(one, batch[i])


@pytest.mark.parametrize("nside,lmax,nsweeps", [(16, 32, 140), (32, 64, 12), (64, 128, 6),
                                                (128, 256, 4), (256, 512, 2)])
def test_solve_parity(torch_dev, nside, lmax, nsweeps):
    torch = torch_dev
    _log("solve parity", nside, lmax, nsweeps)
    c = small_band_inputs(nside, lmax, seed=1)
    lams = c["schedule"] if nsweeps == len(c["schedule"]) else np.geomspace(1e4, 1.0, nsweeps)
    with _plan(nside, lmax, cl=c["cl"], ninv=c["ninv"]) as p:
        s_wf, s_alm = p.solve(torch.from_numpy(c["d"]).cuda(), lams)
        torch.cuda.synchronize()
        p.sync()
        ref_map, ref_alm = messenger.solve(c["d"], c["ninv"], c["cl"], lams, nside, lmax)
        e_map = rel_l2(s_wf.cpu().numpy(), ref_map)
        e_alm = alm_rel_l2(s_alm.cpu().numpy(), ref_alm, lmax)
        _log("  s_wf err", e_map, "alm err", e_alm)
        assert e_map <= SOLVE_TOL
        assert e_alm <= SOLVE_TOL


def test_solve_batch_matches_single(torch_dev):
    torch = torch_dev
    nside, lmax = 32, 64
    cs = [small_band_inputs(nside, lmax, seed=s) for s in range(3)]
    lams = np.geomspace(100.0, 1.0, 5)
    d = np.stack([c["d"] for c in cs])
    with _plan(nside, lmax, cl=cs[0]["cl"], ninv=cs[0]["ninv"], max_batch=3) as p:
        sb, ab = p.solve(torch.from_numpy(d).cuda(), lams)
        for i in range(3):
            s1, a1 = p.solve(torch.from_numpy(d[i].copy()).cuda(), lams)
            assert np.array_equal(s1.cpu().numpy(), sb[i].cpu().numpy())
            assert np.array_equal(a1.cpu().numpy(), ab[i].cpu().numpy())
